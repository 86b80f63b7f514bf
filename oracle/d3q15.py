"""FP64 CPU oracle for the D3Q15 MRT + absorbing-layer step (the paper's
three-dimensional transform matrix, Appendix A.2).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module. It shares no code
with the HIP path (``paper_1203_6350_amd``) and neither imports the other.

Layout: ``f[15][nz][ny][nx]`` (x fastest); velocity order of the columns of
M's rows 1-3: c0 = 0, c1,2 = +-x, c3,4 = +-y, c5,6 = +-z, c7..14 = the
diagonals (+-1, +-1, +-1) with x varying fastest, then y, then z.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm3_oracle.c")
_LIB = os.path.join(_HERE, "liboracle3.so")

VARIANTS = {"none": 0, "I": 1, "II": 2, "III": 3, "visc": 4}
# MRT keeps the four conserved rates at 0; the others share one value here
S3_DEFAULT = (0.0, 0.0, 0.0, 0.0) + (1.9,) * 11


def build(force: bool = False) -> str:
    """Compile lbm3_oracle.c with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # the mutation tests point this at a deliberately broken copy
        alt = os.environ.get("LBM_ORACLE3_LIB")
        L = ctypes.CDLL(alt if alt else build())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i64 = ctypes.c_int64
        L.oracle3_step.argtypes = [i64, i64, i64, dp, dp, dp, dp, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, i64, ctypes.c_int]
        L.oracle3_step.restype = ctypes.c_int
        L.oracle3_feq_field.argtypes = [i64, dp, dp, dp, dp, dp]
        L.oracle3_feq_field.restype = ctypes.c_int
        L.oracle3_collide.argtypes = [i64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, dp]
        L.oracle3_collide.restype = ctypes.c_int
        L.oracle3_tables.argtypes = [dp, dp, ip, ip, ip, dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tables():
    """(M, M^-1, cx, cy, cz, w)."""
    m = np.empty((15, 15))
    mi = np.empty((15, 15))
    c = [np.empty(15, dtype=np.int32) for _ in range(3)]
    w = np.empty(15)
    ip = ctypes.POINTER(ctypes.c_int)
    lib().oracle3_tables(_dp(m), _dp(mi), c[0].ctypes.data_as(ip), c[1].ctypes.data_as(ip),
                         c[2].ctypes.data_as(ip), _dp(w))
    return m, mi, c[0], c[1], c[2], w


def feq_field(rho, ux, uy, uz):
    rho, ux, uy, uz = (_f64(np.broadcast_to(a, np.shape(rho))) for a in (rho, ux, uy, uz))
    out = np.empty((15,) + rho.shape)
    lib().oracle3_feq_field(rho.size, _dp(rho), _dp(ux), _dp(uy), _dp(uz), _dp(out))
    return out


def step(f, nsteps, *, s=S3_DEFAULT, chi=None, qref=(1.0, 0.0, 0.0, 0.0), n=0.5, m=0.5,
         variant="II", nthreads=0):
    """Advance ``f[15][nz][ny][nx]`` by ``nsteps`` steps; returns a new array."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.ndim == 4 and f.shape[0] == 15
    nz, ny, nx = f.shape[1:]
    chi_a = None if chi is None else _f64(np.broadcast_to(chi, (nz, ny, nx)))
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rc = lib().oracle3_step(nx, ny, nz, _dp(f), _dp(chi_a), _dp(_f64(qref)), _dp(_f64(s)),
                            float(n), float(m), v, int(nsteps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle3_step rejected its arguments")
    return f


def collide(fin, *, s=S3_DEFAULT, chi=0.0, qref=(1.0, 0.0, 0.0, 0.0), n=0.5, m=0.5,
            variant="II"):
    """One collision of independent cells: fin [ncell][15] -> [ncell][15]."""
    fin = _f64(fin)
    nc = fin.shape[0]
    out = np.empty_like(fin)
    ch = _f64(np.broadcast_to(chi, (nc,)))
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rc = lib().oracle3_collide(nc, _dp(fin), _dp(ch), _dp(_f64(qref)), _dp(_f64(s)), float(n),
                               float(m), v, _dp(out))
    if rc != 0:
        raise ValueError("oracle3_collide rejected its arguments")
    return out


def moments(f):
    """rho = sum f, u = sum c f / rho."""
    _, _, cx, cy, cz, _ = tables()
    rho = f.sum(axis=0)
    j = [np.tensordot(c.astype(np.float64), f, axes=(0, 0)) for c in (cx, cy, cz)]
    return rho, j[0] / rho, j[1] / rho, j[2] / rho
