"""ctypes loader and build step for the plain C + OpenMP fp64 oracle.

TEST INFRASTRUCTURE (see the package docstring).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "stag_oracle.c")
LIB = os.path.join(_HERE, "c", "liboracle.so")

# Portable x86-64 code (the library may run on a different host CPU than the
# one it was built on); no FMA contraction so the arithmetic is the plain
# sequence of the source.
CFLAGS = ["-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        l = ctypes.CDLL(LIB)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.c_void_p
        l.oracle_threads.restype = ctypes.c_int
        l.oracle_dslash.argtypes = [ip, dp, dp, dp, dp, ctypes.c_int]
        l.oracle_apply_A.argtypes = [ip, dp, dp, ctypes.c_double, dp, dp]
        l.oracle_cg.argtypes = [ip, dp, ctypes.c_double, dp, dp, ctypes.c_double,
                                ctypes.c_long, ctypes.POINTER(ctypes.c_long),
                                ctypes.POINTER(ctypes.c_double)]
        l.oracle_cg_fixed.argtypes = [ip, dp, ctypes.c_double, dp, dp, ctypes.c_long]
        _lib = l
    return _lib


def _L(L):
    return (ctypes.c_int * 4)(*[int(v) for v in L])


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def threads() -> int:
    return int(lib().oracle_threads())


def dslash(U, v, L, p_in, Ulong=None):
    """D of Eq.5 (Ulong: the improved operator, U = fat links)."""
    U = _c128(U)
    v = _c128(v)
    N = None if Ulong is None else _c128(Ulong)
    out = np.empty_like(v)
    rc = lib().oracle_dslash(_L(L), U.ctypes.data, None if N is None else N.ctypes.data,
                             v.ctypes.data, out.ctypes.data, int(p_in))
    if rc:
        raise ValueError(f"oracle_dslash failed ({rc})")
    return out


def apply_A(U, v, L, m, Ulong=None):
    """A = m^2 - D_eo D_oe on even vectors (Ulong: the improved operator)."""
    U = _c128(U)
    v = _c128(v)
    N = None if Ulong is None else _c128(Ulong)
    out = np.empty_like(v)
    rc = lib().oracle_apply_A(_L(L), U.ctypes.data, None if N is None else N.ctypes.data,
                              float(m), v.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError(f"oracle_apply_A failed ({rc})")
    return out


def cg(U, b, L, m, tol, max_iter=0):
    U = _c128(U)
    b = _c128(b)
    x = np.empty_like(b)
    it = ctypes.c_long(0)
    tr = ctypes.c_double(0.0)
    rc = lib().oracle_cg(_L(L), U.ctypes.data, float(m), b.ctypes.data, x.ctypes.data,
                         float(tol), int(max_iter), ctypes.byref(it), ctypes.byref(tr))
    if rc < 0:
        raise ValueError(f"oracle_cg failed ({rc})")
    status = {0: "ok", 1: "noconv", 2: "breakdown"}[rc]
    return x, dict(iters=int(it.value), true_rel_res=float(tr.value), status=status)


def cg_fixed(U, b, L, m, n_iter):
    """Exactly n_iter Fig.1 iterations (a bounded timing sample)."""
    U = _c128(U)
    b = _c128(b)
    x = np.empty_like(b)
    rc = lib().oracle_cg_fixed(_L(L), U.ctypes.data, float(m), b.ctypes.data, x.ctypes.data,
                               int(n_iter))
    if rc:
        raise ValueError(f"oracle_cg_fixed failed ({rc})")
    return x
