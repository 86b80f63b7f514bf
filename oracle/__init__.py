"""FP64 CPU oracle for the D2Q9 MRT + absorbing-layer lattice Boltzmann step.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the HIP path (``paper_1203_6350_amd``) and neither imports the other.

Two independent implementations live here:

* ``lbm_oracle.c`` (O1): the time stepper, plain C in FP64, dense transform
  matrix M (Appendix A.1), velocity-space equilibria, damping term of
  eq. blbs-abc-1 with Gamma = chi I (eq. eq:gamma) for the Types I, II and III
  of Sections 2.2.1-2.2.3, and a separate periodic streaming pass.
* ``vn.py`` (O2): the Von Neumann analysis of Section 3.2 in numpy, with its
  own copy of the collision written for complex arithmetic.

``lbm_oracle.c`` also holds the diagnostics (the density and momentum
deviations whose L2 norm Section 4.1 tracks, the largest population
deviation over the finite cells, the count of non-finite cells).

Population layout everywhere: ``f[9][ny][nx]`` (x fastest), velocity order of
M's columns: c0=(0,0) c1=(1,0) c2=(0,1) c3=(-1,0) c4=(0,-1) c5=(1,1)
c6=(-1,1) c7=(-1,-1) c8=(1,-1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

VARIANTS = {"none": 0, "I": 1, "II": 2, "III": 3, "I_rewritten": 4, "visc": 5}

# Default relaxation rates: s = 1.9 is the only value stated in prose for the
# Von Neumann study (Section 3.3); MRT keeps S(0..2) = 0 (Section 2.1).
S_MRT_DEFAULT = (0.0, 0.0, 0.0, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9)


def build(force: bool = False) -> str:
    """Compile lbm_oracle.c with gcc (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # the mutation tests point this at a deliberately broken copy
        alt = os.environ.get("LBM_ORACLE_LIB")
        if alt:
            L = ctypes.CDLL(alt)
        else:
            build()
            L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_step.argtypes = [i64, i64, dp, dp, dp, dp, dp, dp,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                  i64, ctypes.c_int]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step_avg.argtypes = [i64, i64, dp, dp, dp, dp, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_double, i64,
                                      ctypes.c_int]
        L.oracle_step_avg.restype = ctypes.c_int
        L.oracle_step_line_source.argtypes = [i64, i64, dp, dp, dp, dp, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, dp, ctypes.c_int,
                                              i64, i64, ctypes.c_int]
        L.oracle_step_line_source.restype = ctypes.c_int
        L.oracle_collide.argtypes = [i64, dp, dp, dp, dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, dp]
        L.oracle_collide.restype = ctypes.c_int
        L.oracle_feq_field.argtypes = [i64, dp, dp, dp, dp]
        L.oracle_flin_field.argtypes = [i64, dp, dp, dp, dp]
        L.oracle_tables.argtypes = [dp, dp, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), dp]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_diagnostics.argtypes = [i64, i64, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, dp]
        L.oracle_diagnostics.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def tables():
    """(M, M^-1, cx, cy, w) exactly as the oracle holds them."""
    M = np.zeros((9, 9))
    Mi = np.zeros((9, 9))
    cx = np.zeros(9, dtype=np.int32)
    cy = np.zeros(9, dtype=np.int32)
    w = np.zeros(9)
    lib().oracle_tables(_dp(M), _dp(Mi), cx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        cy.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    return M, Mi, cx, cy, w


def feq_field(rho, ux, uy):
    """Equilibrium f^eq(rho, u) for fields of any shape -> [9, *shape]."""
    rho = _f64(rho)
    shape = rho.shape
    ux = _f64(np.broadcast_to(ux, shape))
    uy = _f64(np.broadcast_to(uy, shape))
    out = np.empty((9,) + shape)
    lib().oracle_feq_field(rho.size, _dp(rho), _dp(ux), _dp(uy), _dp(out))
    return out


def flin_field(rho, ux, uy):
    rho = _f64(rho)
    shape = rho.shape
    ux = _f64(np.broadcast_to(ux, shape))
    uy = _f64(np.broadcast_to(uy, shape))
    out = np.empty((9,) + shape)
    lib().oracle_flin_field(rho.size, _dp(rho), _dp(ux), _dp(uy), _dp(out))
    return out


def step(f, nsteps, *, s=S_MRT_DEFAULT, chi=None, qref=(1.0, 0.0, 0.0),
         qref_field=None, srel=None, n=0.5, m=0.5, variant="II", nthreads=0):
    """Advance pre-collision populations ``f[9][ny][nx]`` by ``nsteps`` steps.

    Returns a new array; the input is not modified.
    """
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.ndim == 3 and f.shape[0] == 9
    ny, nx = f.shape[1:]
    chi_a = None if chi is None else _f64(np.broadcast_to(chi, (ny, nx)))
    qf = None if qref_field is None else _f64(qref_field).reshape(3, ny, nx)
    qu = _f64(qref)
    sr = None if srel is None else _f64(np.broadcast_to(srel, (ny, nx)))
    sv = _f64(s)
    assert sv.shape == (9,)
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rc = lib().oracle_step(nx, ny, _dp(f), _dp(chi_a), _dp(qf), _dp(qu), _dp(sv),
                           _dp(sr), float(n), float(m), v, int(nsteps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_step rejected its arguments")
    return f


def step_avg(f, cf, nsteps, *, alpha, s=S_MRT_DEFAULT, chi=None, n=0.5, m=0.5, variant="II",
             nthreads=0):
    """Advance ``f[9][ny][nx]`` by ``nsteps`` steps with a time-averaged
    reference state ``cf[3][ny][nx]`` = (rho^f, j^f_x, j^f_y): every step
    collides with q_ref = (rho^f, j^f / rho^f), then c^f += alpha (c - c^f)
    with the cell's pre-collision moments c (Sec. 1, Sec. 2.2).

    Returns (f, cf), new arrays.
    """
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.ndim == 3 and f.shape[0] == 9
    ny, nx = f.shape[1:]
    cf = np.array(np.broadcast_to(cf, (3, ny, nx)), dtype=np.float64, order="C", copy=True)
    chi_a = None if chi is None else _f64(np.broadcast_to(chi, (ny, nx)))
    sv = _f64(s)
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rc = lib().oracle_step_avg(nx, ny, _dp(f), _dp(chi_a), _dp(cf), _dp(sv), float(n), float(m),
                               v, float(alpha), int(nsteps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_step_avg rejected its arguments")
    return f, cf


def step_line_source(f, nsteps, *, source, outflow=True, t0=0, s=S_MRT_DEFAULT, chi=None,
                     qref=(1.0, 0.0, 0.0), n=0.5, m=0.5, variant="II", nthreads=0):
    """Advance ``f[9][ny][nx]`` by ``nsteps`` steps on the line-source channel
    of Sec. 4.2: after each collision the column x = 0 becomes
    f^eq(rho_src(t + 1), u_src) with rho_src(t) = rho0 + amp sin(2 pi freq t +
    phase), and (outflow) the column x = nx - 1 a copy of column nx - 2.

    ``source`` = (rho0, amp, freq, phase, ux, uy); ``t0`` = step index of
    the input state. Returns a new array.
    """
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.ndim == 3 and f.shape[0] == 9
    ny, nx = f.shape[1:]
    chi_a = None if chi is None else _f64(np.broadcast_to(chi, (ny, nx)))
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rc = lib().oracle_step_line_source(nx, ny, _dp(f), _dp(chi_a), _dp(_f64(qref)), _dp(_f64(s)),
                                       float(n), float(m), v, _dp(_f64(source)), int(bool(outflow)),
                                       int(t0), int(nsteps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_step_line_source rejected its arguments")
    return f


def collide(fin, *, s=S_MRT_DEFAULT, chi=0.0, qref=(1.0, 0.0, 0.0), n=0.5,
            m=0.5, variant="II"):
    """Collision only (no streaming) for independent cells ``fin[ncell][9]``."""
    fin = _f64(fin).reshape(-1, 9)
    nc = fin.shape[0]
    chi_a = _f64(np.broadcast_to(chi, (nc,)))
    q = _f64(np.broadcast_to(np.asarray(qref, dtype=np.float64), (nc, 3)))
    out = np.empty_like(fin)
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rc = lib().oracle_collide(nc, _dp(fin), _dp(chi_a), _dp(q), _dp(_f64(s)),
                              float(n), float(m), v, _dp(out))
    if rc != 0:
        raise ValueError("oracle_collide rejected its arguments")
    return out


def moments(f):
    """Raw moments of pre-collision populations: rho = sum f, u = sum c f / rho."""
    _, _, cx, cy, _ = tables()
    rho = f.sum(axis=0)
    jx = np.tensordot(cx.astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(cy.astype(np.float64), f, axes=(0, 0))
    return rho, jx / rho, jy / rho


def diagnostics(f, rho_b=1.0, ux_b=0.0, uy_b=0.0):
    """Monitored quantities of a pre-collision state ``f[9][ny][nx]`` against
    the base state (rho_b, u_b) (the deviations whose L2 norm Section 4.1
    tracks): (sum drho, sum djx, sum djy, sum drho^2, sum |dj|^2,
    max over finite cells of |f - f^eq(rho_b, u_b)|, non-finite cell count).
    """
    f = _f64(f)
    assert f.ndim == 3 and f.shape[0] == 9
    ny, nx = f.shape[1:]
    out = np.empty(7)
    rc = lib().oracle_diagnostics(nx, ny, _dp(f), float(rho_b), float(ux_b), float(uy_b),
                                  _dp(out))
    if rc != 0:
        raise ValueError("oracle_diagnostics rejected its arguments")
    return out


def max_threads():
    return int(lib().oracle_max_threads())
