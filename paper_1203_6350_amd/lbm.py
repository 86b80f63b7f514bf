"""ctypes binding of liblbm.so (include/lbm.h): the same entry points under
the same names, with numpy arrays marshalled to host pointers and torch
tensors (or raw integers) to device pointers and streams.

There is no fallback: if the HIP library or a gfx950 device is missing every
call raises ``LbmError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
VARIANT = {"none": 0, "I": 1, "II": 2, "III": 3, "visc": 4}
COMBINE = {"max": 0, "sum": 1}
_CODE_NAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSTABLE", -5: "ESTATE"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_CODE_NAMES.get(code, code), msg))
        self.code = code


class LbmUnstable(LbmError):
    """LBM_EUNSTABLE: the instability detector has tripped. The call still
    completed; ``result`` holds what it returns otherwise (or None)."""

    def __init__(self, code, msg, result=None):
        super().__init__(code, msg)
        self.result = result


class lbm_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("rho_base", ctypes.c_double), ("ux_base", ctypes.c_double),
                ("uy_base", ctypes.c_double), ("s", ctypes.c_double * 9),
                ("shift_n", ctypes.c_double), ("shift_m", ctypes.c_double),
                ("storage", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("f16_scale", ctypes.c_double), ("stream", ctypes.c_void_p)]


class lbm_qref(ctypes.Structure):
    _fields_ = [("rho_f", ctypes.c_double), ("ux_f", ctypes.c_double), ("uy_f", ctypes.c_double)]


class lbm_info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("pitch", ctypes.c_int64),
                ("plane_stride", ctypes.c_int64), ("steps_done", ctypes.c_int64),
                ("storage", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("elem_bytes", ctypes.c_int32), ("chi_mode", ctypes.c_int32),
                ("device_bytes", ctypes.c_size_t)]


class lbm_line_source(ctypes.Structure):
    _fields_ = [("rho0", ctypes.c_double), ("amp", ctypes.c_double), ("freq", ctypes.c_double),
                ("phase", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double)]


class lbm_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("block", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("rows", ctypes.c_int32)]

    def as_dict(self):
        return {"kernel": self.kernel, "block": self.block, "nontemporal": self.nontemporal,
                "rows": self.rows}


class lbm3_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("rho_base", ctypes.c_double), ("ux_base", ctypes.c_double),
                ("uy_base", ctypes.c_double), ("uz_base", ctypes.c_double),
                ("s", ctypes.c_double * 15),
                ("shift_n", ctypes.c_double), ("shift_m", ctypes.c_double),
                ("storage", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("f16_scale", ctypes.c_double), ("stream", ctypes.c_void_p)]


class lbm3_qref(ctypes.Structure):
    _fields_ = [("rho_f", ctypes.c_double), ("ux_f", ctypes.c_double), ("uy_f", ctypes.c_double),
                ("uz_f", ctypes.c_double)]


class lbm_vn_params(ctypes.Structure):
    _fields_ = [("s", ctypes.c_double * 9), ("shift_n", ctypes.c_double),
                ("shift_m", ctypes.c_double), ("chi", ctypes.c_double),
                ("rho_f", ctypes.c_double), ("ux_f", ctypes.c_double),
                ("uy_f", ctypes.c_double), ("variant", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p


def load(path: str | None = None):
    """Load liblbm.so (torch is imported first so that both share one HIP
    runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (brings the process's HIP runtime)
    except Exception:
        pass
    p = path or os.environ.get("LBM_LIB", LIB_PATH)
    if not os.path.exists(p):
        raise LbmError(LBM_EDEVICE, "liblbm.so not built at %s (run __graft_entry__.build())" % p)
    L = ctypes.CDLL(p)
    i64, i32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "lbm_create": [ctypes.POINTER(lbm_config), _DP, _DP, _DP, ctypes.POINTER(_H)],
        "lbm_required_bytes": [ctypes.POINTER(lbm_config), ctypes.POINTER(sz)],
        "lbm_create_ext": [ctypes.POINTER(lbm_config), _DP, _DP, _DP, vp, vp, sz, ctypes.POINTER(_H)],
        "lbm_set_sponge": [_H, _DP, ctypes.POINTER(lbm_qref)],
        "lbm_set_sponge_separable": [_H, _DP, _DP, i32, ctypes.POINTER(lbm_qref)],
        "lbm_set_sponge_separable_dev": [_H, vp, vp, i32, ctypes.POINTER(lbm_qref)],
        "lbm_step": [_H, i64],
        "lbm_sync": [_H],
        "lbm_moments": [_H, _DP, _DP, _DP],
        "lbm_moments_dev": [_H, vp, vp, vp],
        "lbm_diagnostics": [_H, _DP],
        "lbm_diagnostics_dev": [_H, vp],
        "lbm_diagnostics_dev_noalloc": [_H, vp],
        "lbm_get_populations": [_H, _DP],
        "lbm_set_populations": [_H, _DP],
        "lbm_get_info": [_H, ctypes.POINTER(lbm_info)],
        "lbm_set_tuning": [_H, ctypes.POINTER(lbm_tuning)],
        "lbm_set_qref_field": [_H, _DP, _DP, _DP],
        "lbm_set_line_source": [_H, ctypes.POINTER(lbm_line_source), i32],
        "lbm_set_qref_average": [_H, ctypes.c_double],
        "lbm_get_qref_field": [_H, _DP, _DP, _DP],
        "lbm_get_tuning": [_H, ctypes.POINTER(lbm_tuning)],
        "lbm_autotune": [_H, i32, ctypes.POINTER(lbm_tuning), _DP],
        "lbm_state_bytes": [_H, ctypes.POINTER(sz)],
        "lbm_save_state": [_H, vp, sz],
        "lbm_load_state": [_H, vp, sz],
        "vn_amplification": [ctypes.POINTER(lbm_vn_params), i64, _DP, _DP, _DP, _DP],
        "vn_amplification_dev": [ctypes.POINTER(lbm_vn_params), i64, i64, vp, vp, vp, vp, vp],
        "lbm_device_copy": [vp, vp, sz, vp],
        "lbm_batch_create": [ctypes.POINTER(_H), i32, vp, ctypes.POINTER(_H)],
        "lbm_batch_step": [_H, i64],
        "lbm_batch_tick": [_H, i32, ctypes.POINTER(ctypes.c_int32)],
        "lbm_batch_set_grid": [_H, i32],
        "lbm_batch_set_tuning": [_H, ctypes.POINTER(lbm_tuning)],
        "lbm_batch_get_tuning": [_H, ctypes.POINTER(lbm_tuning)],
        "lbm_batch_set_min_items": [_H, i32],
        "lbm_batch_set_members": [_H, ctypes.POINTER(_H), i32],
        "lbm_init_fields_dev": [_H, vp, vp, vp],
        "lbm_batch_sync": [_H],
        "lbm_set_detector": [_H, i64, ctypes.c_double],
        "lbm_detector_status": [_H, ctypes.POINTER(i64)],
        "lbm_batch_detector_status": [_H, ctypes.POINTER(i64)],
        "lbm3_create": [ctypes.POINTER(lbm3_config), _DP, _DP, _DP, _DP, ctypes.POINTER(_H)],
        "lbm3_set_sponge": [_H, _DP, ctypes.POINTER(lbm3_qref)],
        "lbm3_set_sponge_separable": [_H, _DP, _DP, _DP, i32, ctypes.POINTER(lbm3_qref)],
        "lbm3_step": [_H, i64],
        "lbm3_sync": [_H],
        "lbm3_get_populations": [_H, _DP],
        "lbm3_set_populations": [_H, _DP],
        "lbm3_moments": [_H, _DP, _DP, _DP, _DP],
        "lbm3_steps_done": [_H, ctypes.POINTER(i64)],
        "lbm3_set_tuning": [_H, i32, i32],
        "lbm3_get_tuning": [_H, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "lbm3_autotune": [_H, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), _DP],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.lbm_destroy.argtypes = [_H]
    L.lbm_destroy.restype = None
    L.lbm_batch_destroy.argtypes = [_H]
    L.lbm_batch_destroy.restype = None
    L.lbm3_destroy.argtypes = [_H]
    L.lbm3_destroy.restype = None
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc, result=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error()
        msg = msg.decode() if msg else ""
        if rc == LBM_EUNSTABLE:
            raise LbmUnstable(rc, msg, result)
        raise LbmError(rc, msg)


def _host(a, n=None):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and arr.size != n:
        raise ValueError("expected %d values, got %d" % (n, arr.size))
    return arr, arr.ctypes.data_as(_DP)


def _dev(t):
    """Device pointer of a torch tensor, an int address, or None."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def make_config(nx, ny, *, s=(0, 0, 0, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9), storage="f32",
                variant="II", rho_base=1.0, ux_base=0.0, uy_base=0.0, shift_n=0.5,
                shift_m=0.5, f16_scale=1e-3, stream=None):
    c = lbm_config()
    c.nx, c.ny = int(nx), int(ny)
    c.rho_base, c.ux_base, c.uy_base = float(rho_base), float(ux_base), float(uy_base)
    for k in range(9):
        c.s[k] = float(s[k])
    c.shift_n, c.shift_m = float(shift_n), float(shift_m)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.variant = VARIANT[variant] if isinstance(variant, str) else int(variant)
    c.f16_scale = float(f16_scale)
    c.stream = _stream_ptr(stream)
    return c


# ---------------------------------------------------------------- entry points

def lbm_create(cfg, rho=None, ux=None, uy=None):
    L = load()
    n = cfg.nx * cfg.ny
    _r, pr = _host(rho, n)
    _u, pu = _host(ux, n)
    _v, pv = _host(uy, n)
    h = _H()
    _check(L.lbm_create(ctypes.byref(cfg), pr, pu, pv, ctypes.byref(h)))
    return h


def lbm_required_bytes(cfg):
    b = ctypes.c_size_t()
    _check(load().lbm_required_bytes(ctypes.byref(cfg), ctypes.byref(b)))
    return b.value


def lbm_create_ext(cfg, buf_a, buf_b, rho=None, ux=None, uy=None):
    """Create on caller-owned device buffers (e.g. torch uint8 tensors)."""
    L = load()
    n = cfg.nx * cfg.ny
    _r, pr = _host(rho, n)
    _u, pu = _host(ux, n)
    _v, pv = _host(uy, n)
    each = min(buf_a.numel() * buf_a.element_size(), buf_b.numel() * buf_b.element_size())
    h = _H()
    _check(L.lbm_create_ext(ctypes.byref(cfg), pr, pu, pv, _dev(buf_a), _dev(buf_b), each,
                            ctypes.byref(h)))
    return h


def _qref(q):
    if q is None:
        return None
    qq = lbm_qref(float(q[0]), float(q[1]), float(q[2]))
    return ctypes.byref(qq)


def lbm_set_sponge(h, chi=None, qref=None, *, nx=None, ny=None):
    _c, pc = _host(chi)
    _check(load().lbm_set_sponge(h, pc, _qref(qref)))


def lbm_set_sponge_separable(h, chi_x=None, chi_y=None, combine="max", qref=None):
    _a, pa = _host(chi_x)
    _b, pb = _host(chi_y)
    cm = COMBINE[combine] if isinstance(combine, str) else int(combine)
    _check(load().lbm_set_sponge_separable(h, pa, pb, cm, _qref(qref)))


def lbm_set_sponge_separable_dev(h, chi_x=None, chi_y=None, combine="max", qref=None):
    """Separable sponge from FP64 device tensors (or addresses); stream-ordered,
    not validated."""
    _check(load().lbm_set_sponge_separable_dev(h, _dev(chi_x), _dev(chi_y), COMBINE[combine],
                                               _qref(qref)))


def lbm_step(h, n=1):
    _check(load().lbm_step(h, int(n)))


def lbm_sync(h):
    _check(load().lbm_sync(h))


def lbm_get_info(h):
    info = lbm_info()
    _check(load().lbm_get_info(h, ctypes.byref(info)))
    return info


def lbm_set_qref_field(h, rho_f=None, ux_f=None, uy_f=None):
    """Per-cell reference state (host arrays [ny][nx]); all None clears it."""
    info = lbm_get_info(h) if rho_f is not None else None
    n = None if info is None else info.nx * info.ny
    _r, pr = _host(rho_f, n)
    _u, pu = _host(ux_f, n)
    _v, pv = _host(uy_f, n)
    _check(load().lbm_set_qref_field(h, pr, pu, pv))


def lbm_set_line_source(h, source=None, outflow=True):
    """source = (rho0, amp, freq, phase, ux, uy) or None (periodic x again)."""
    if source is None:
        _check(load().lbm_set_line_source(h, None, 0))
        return
    src = lbm_line_source(*(float(v) for v in source))
    _check(load().lbm_set_line_source(h, ctypes.byref(src), int(bool(outflow))))


def lbm_set_qref_average(h, alpha):
    _check(load().lbm_set_qref_average(h, float(alpha)))


def lbm_get_qref_field(h):
    info = lbm_get_info(h)
    shape = (info.ny, info.nx)
    rho, ux, uy = (np.empty(shape) for _ in range(3))
    _check(load().lbm_get_qref_field(h, rho.ctypes.data_as(_DP), ux.ctypes.data_as(_DP),
                                     uy.ctypes.data_as(_DP)))
    return rho, ux, uy


def lbm_moments(h):
    info = lbm_get_info(h)
    shape = (info.ny, info.nx)
    rho, ux, uy = (np.empty(shape) for _ in range(3))
    _check(load().lbm_moments(h, rho.ctypes.data_as(_DP), ux.ctypes.data_as(_DP),
                              uy.ctypes.data_as(_DP)), (rho, ux, uy))
    return rho, ux, uy


def lbm_moments_dev(h, rho, ux, uy):
    _check(load().lbm_moments_dev(h, _dev(rho), _dev(ux), _dev(uy)))


def lbm_diagnostics(h):
    out = np.empty(7)
    _check(load().lbm_diagnostics(h, out.ctypes.data_as(_DP)), out)
    return out


def lbm_set_detector(h, every_n, max_dev=float("inf")):
    """Instability detector: check every ``every_n`` steps (0: off) for
    non-finite populations or deviations above ``max_dev``."""
    _check(load().lbm_set_detector(h, int(every_n), float(max_dev)))


def lbm_detector_status(h):
    """Step count of the detector's first trip, or -1."""
    t = ctypes.c_int64(-1)
    _check(load().lbm_detector_status(h, ctypes.byref(t)))
    return int(t.value)


def lbm_diagnostics_dev(h, out7):
    _check(load().lbm_diagnostics_dev(h, _dev(out7)))


def lbm_diagnostics_dev_noalloc(h, out7):
    """lbm_diagnostics_dev with its partials in the library's static device
    workspace (no allocation; overlapping calls on one device race)."""
    _check(load().lbm_diagnostics_dev_noalloc(h, _dev(out7)))


def lbm_get_populations(h):
    info = lbm_get_info(h)
    f = np.empty((9, info.ny, info.nx))
    _check(load().lbm_get_populations(h, f.ctypes.data_as(_DP)))
    return f


def lbm_set_populations(h, f):
    info = lbm_get_info(h)
    _a, pa = _host(f, 9 * info.nx * info.ny)
    _check(load().lbm_set_populations(h, pa))


def lbm_set_tuning(h, kernel=1, block=256, nontemporal=0, rows=0):
    t = lbm_tuning(int(kernel), int(block), int(nontemporal), int(rows))
    _check(load().lbm_set_tuning(h, ctypes.byref(t)))


def lbm_get_tuning(h):
    t = lbm_tuning()
    _check(load().lbm_get_tuning(h, ctypes.byref(t)))
    return t.as_dict()


def lbm_autotune(h, reps=10):
    t = lbm_tuning()
    ms = ctypes.c_double()
    _check(load().lbm_autotune(h, int(reps), ctypes.byref(t), ctypes.byref(ms)))
    return t.as_dict(), ms.value


def lbm_state_bytes(h):
    b = ctypes.c_size_t()
    _check(load().lbm_state_bytes(h, ctypes.byref(b)))
    return b.value


def lbm_save_state(h):
    buf = np.empty(lbm_state_bytes(h), dtype=np.uint8)
    _check(load().lbm_save_state(h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
    return buf


def lbm_load_state(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(load().lbm_load_state(h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))


def lbm_destroy(h):
    if h is not None and load() is not None:
        load().lbm_destroy(h)


def lbm_last_error():
    m = load().lbm_last_error()
    return m.decode() if m else ""


def _vn_params(p):
    v = lbm_vn_params()
    for k in range(9):
        v.s[k] = float(p["s"][k])
    v.shift_n = float(p.get("n", 0.5))
    v.shift_m = float(p.get("m", 0.5))
    v.chi = float(p["chi"])
    q = p.get("qref", (1.0, 0.0, 0.0))
    v.rho_f, v.ux_f, v.uy_f = float(q[0]), float(q[1]), float(q[2])
    var = p.get("variant", "II")
    v.variant = VARIANT[var] if isinstance(var, str) else int(var)
    return v


def vn_amplification(params, kx, ky, want_G=False):
    """Eigenvalues (nk, 9) complex, sorted by (-|lambda|, arg), and optionally
    G (nk, 9, 9) complex, for one parameter set (dict with s, chi, qref,
    variant, n, m)."""
    L = load()
    kx = np.ascontiguousarray(kx, dtype=np.float64).ravel()
    ky = np.ascontiguousarray(ky, dtype=np.float64).ravel()
    nk = kx.size
    eig = np.empty((nk, 9, 2))
    G = np.empty((nk, 9, 9, 2)) if want_G else None
    v = _vn_params(params)
    _check(L.vn_amplification(ctypes.byref(v), nk, kx.ctypes.data_as(_DP), ky.ctypes.data_as(_DP),
                              eig.ctypes.data_as(_DP), G.ctypes.data_as(_DP) if want_G else None))
    lam = eig[..., 0] + 1j * eig[..., 1]
    if want_G:
        return lam, G[..., 0] + 1j * G[..., 1]
    return lam


def vn_amplification_dev(param_list, kx, ky, eig, G=None, stream=None):
    """Batched device form: kx, ky (nk,) float64 tensors; eig
    (nparams, nk, 9, 2) float64 tensor; G optional (nparams, nk, 9, 9, 2)."""
    arr = (lbm_vn_params * len(param_list))(*[_vn_params(p) for p in param_list])
    _check(load().vn_amplification_dev(arr, len(param_list), int(kx.numel()), _dev(kx), _dev(ky),
                                       _dev(eig), _dev(G), _stream_ptr(stream)))


def lbm_device_copy(dst, src, nbytes, stream=None):
    _check(load().lbm_device_copy(_dev(dst), _dev(src), int(nbytes), _stream_ptr(stream)))


# ---------------------------------------------------------------- convenience

class Lattice:
    """Owning wrapper of one lattice handle."""

    def __init__(self, nx, ny, *, rho=None, ux=None, uy=None, **cfg_kw):
        self.cfg = make_config(nx, ny, **cfg_kw)
        self.h = lbm_create(self.cfg, rho, ux, uy)
        self.nx, self.ny = int(nx), int(ny)

    def set_sponge(self, chi=None, qref=None):
        lbm_set_sponge(self.h, chi, qref)

    def set_sponge_separable(self, chi_x=None, chi_y=None, combine="max", qref=None):
        lbm_set_sponge_separable(self.h, chi_x, chi_y, combine, qref)

    def step(self, n=1):
        lbm_step(self.h, n)

    def sync(self):
        lbm_sync(self.h)

    def moments(self):
        return lbm_moments(self.h)

    def set_qref_field(self, rho_f=None, ux_f=None, uy_f=None):
        lbm_set_qref_field(self.h, rho_f, ux_f, uy_f)

    def set_qref_average(self, alpha):
        lbm_set_qref_average(self.h, alpha)

    def set_line_source(self, source=None, outflow=True):
        lbm_set_line_source(self.h, source, outflow)

    def qref_field(self):
        return lbm_get_qref_field(self.h)

    def diagnostics(self):
        return lbm_diagnostics(self.h)

    def set_detector(self, every_n, max_dev=float("inf")):
        lbm_set_detector(self.h, every_n, max_dev)

    def detector_status(self):
        return lbm_detector_status(self.h)

    def populations(self):
        return lbm_get_populations(self.h)

    def set_populations(self, f):
        lbm_set_populations(self.h, f)

    def info(self):
        return lbm_get_info(self.h)

    def set_tuning(self, **kw):
        lbm_set_tuning(self.h, **kw)

    def tuning(self):
        return lbm_get_tuning(self.h)

    def autotune(self, reps=10):
        return lbm_autotune(self.h, reps)

    def save_state(self):
        return lbm_save_state(self.h)

    def load_state(self, buf):
        lbm_load_state(self.h, buf)

    def close(self):
        if self.h is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------- batches

def lbm_batch_create(handles, stream=None):
    arr = (_H * len(handles))(*[h.value if isinstance(h, _H) else h for h in handles])
    b = _H()
    _check(load().lbm_batch_create(arr, len(handles), _stream_ptr(stream), ctypes.byref(b)))
    return b


def lbm_batch_set_members(b, handles):
    arr = (_H * len(handles))(*[h.value if isinstance(h, _H) else h for h in handles])
    _check(load().lbm_batch_set_members(b, arr, len(handles)))


def lbm_init_fields_dev(h, rho=None, ux=None, uy=None):
    _check(load().lbm_init_fields_dev(h, _dev(rho), _dev(ux), _dev(uy)))


def lbm_batch_step(b, n):
    _check(load().lbm_batch_step(b, int(n)))


def lbm_batch_tick(b, tick, member_steps=None):
    ms = None
    if member_steps is not None:
        arr = (ctypes.c_int32 * len(member_steps))(*[int(x) for x in member_steps])
        ms = arr
    _check(load().lbm_batch_tick(b, int(tick), ms))


def lbm_batch_set_tuning(b, kernel=4, block=64, nontemporal=0, rows=0):
    t = lbm_tuning(int(kernel), int(block), int(nontemporal), int(rows))
    _check(load().lbm_batch_set_tuning(b, ctypes.byref(t)))


def lbm_batch_get_tuning(b):
    t = lbm_tuning()
    _check(load().lbm_batch_get_tuning(b, ctypes.byref(t)))
    return t.as_dict()


def lbm_batch_set_min_items(b, min_items):
    _check(load().lbm_batch_set_min_items(b, int(min_items)))


def lbm_batch_set_grid(b, blocks_per_cu):
    _check(load().lbm_batch_set_grid(b, int(blocks_per_cu)))


def lbm_batch_sync(b):
    _check(load().lbm_batch_sync(b))


def lbm_batch_detector_status(b, count):
    """Per member: step count of its detector's first trip, or -1."""
    out = np.empty(count, dtype=np.int64)
    _check(load().lbm_batch_detector_status(b, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def lbm_batch_destroy(b):
    if b is not None:
        load().lbm_batch_destroy(b)


class Batch:
    """Many lattices stepped by one persistent launch per step (HIP graphs).

    The batch keeps references to its member Lattice objects; members must not
    be stepped on their own while the batch has work in flight (``sync()``)."""

    def __init__(self, lattices, stream=None):
        self.members = list(lattices)
        self.b = lbm_batch_create([m.h for m in self.members], stream)

    def step(self, n):
        lbm_batch_step(self.b, n)

    def tick(self, tick, member_steps=None):
        lbm_batch_tick(self.b, tick, member_steps)

    def set_grid(self, blocks_per_cu):
        lbm_batch_set_grid(self.b, blocks_per_cu)

    def set_tuning(self, **kw):
        lbm_batch_set_tuning(self.b, **kw)

    def tuning(self):
        return lbm_batch_get_tuning(self.b)

    def set_min_items(self, min_items):
        lbm_batch_set_min_items(self.b, min_items)

    def set_members(self, lattices):
        lbm_batch_set_members(self.b, [m.h for m in lattices])
        self.members = list(lattices)

    def sync(self):
        lbm_batch_sync(self.b)

    def detector_status(self):
        return lbm_batch_detector_status(self.b, len(self.members))

    def close(self):
        if self.b is not None:
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- D3Q15 (include/lbm3.h)

S3_DEFAULT = (0, 0, 0, 0, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9, 1.9)


def make_config3(nx, ny, nz, *, s=S3_DEFAULT, storage="f32", variant="II", rho_base=1.0,
                 ux_base=0.0, uy_base=0.0, uz_base=0.0, shift_n=0.5, shift_m=0.5,
                 f16_scale=1e-3, stream=None):
    c = lbm3_config()
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.rho_base = float(rho_base)
    c.ux_base, c.uy_base, c.uz_base = float(ux_base), float(uy_base), float(uz_base)
    for k in range(15):
        c.s[k] = float(s[k])
    c.shift_n, c.shift_m = float(shift_n), float(shift_m)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.variant = VARIANT[variant] if isinstance(variant, str) else int(variant)
    c.f16_scale = float(f16_scale)
    c.stream = _stream_ptr(stream)
    return c


def _qref3(q):
    if q is None:
        return None
    return ctypes.byref(lbm3_qref(*[float(v) for v in q]))


def lbm3_create(cfg, rho=None, ux=None, uy=None, uz=None):
    L = load()
    n = cfg.nx * cfg.ny * cfg.nz
    keep = [_host(a, n) for a in (rho, ux, uy, uz)]
    h = _H()
    _check(L.lbm3_create(ctypes.byref(cfg), *[p for _a, p in keep], ctypes.byref(h)))
    return h


def lbm3_set_sponge(h, chi=None, qref=None):
    _c, pc = _host(chi)
    _check(load().lbm3_set_sponge(h, pc, _qref3(qref)))


def lbm3_set_sponge_separable(h, chi_x=None, chi_y=None, chi_z=None, combine="max", qref=None):
    keep = [_host(a) for a in (chi_x, chi_y, chi_z)]
    cm = COMBINE[combine] if isinstance(combine, str) else int(combine)
    _check(load().lbm3_set_sponge_separable(h, *[p for _a, p in keep], cm, _qref3(qref)))


def lbm3_step(h, n=1):
    _check(load().lbm3_step(h, int(n)))


def lbm3_sync(h):
    _check(load().lbm3_sync(h))


def lbm3_get_populations(h, shape):
    nz, ny, nx = shape
    f = np.empty((15, nz, ny, nx), dtype=np.float64)
    _check(load().lbm3_get_populations(h, f.ctypes.data_as(_DP)))
    return f


def lbm3_set_populations(h, f):
    arr = np.ascontiguousarray(f, dtype=np.float64)
    _check(load().lbm3_set_populations(h, arr.ctypes.data_as(_DP)))


def lbm3_moments(h, shape):
    out = [np.empty(shape, dtype=np.float64) for _ in range(4)]
    _check(load().lbm3_moments(h, *[o.ctypes.data_as(_DP) for o in out]))
    return tuple(out)


def lbm3_steps_done(h):
    v = ctypes.c_int64()
    _check(load().lbm3_steps_done(h, ctypes.byref(v)))
    return v.value


def lbm3_set_tuning(h, kernel=0, block=256):
    _check(load().lbm3_set_tuning(h, int(kernel), int(block)))


def lbm3_get_tuning(h):
    k, b = ctypes.c_int32(), ctypes.c_int32()
    _check(load().lbm3_get_tuning(h, ctypes.byref(k), ctypes.byref(b)))
    return {"kernel": k.value, "block": b.value}


def lbm3_autotune(h, reps=5):
    k, b, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load().lbm3_autotune(h, int(reps), ctypes.byref(k), ctypes.byref(b), ctypes.byref(ms)))
    return {"kernel": k.value, "block": b.value}, ms.value


def lbm3_destroy(h):
    load().lbm3_destroy(h)


class Lattice3:
    """Owning wrapper of one D3Q15 lattice handle; host arrays [nz][ny][nx]."""

    def __init__(self, nx, ny, nz, *, rho=None, ux=None, uy=None, uz=None, **cfg_kw):
        self.cfg = make_config3(nx, ny, nz, **cfg_kw)
        self.h = lbm3_create(self.cfg, rho, ux, uy, uz)
        self.shape = (int(nz), int(ny), int(nx))

    def set_sponge(self, chi=None, qref=None):
        lbm3_set_sponge(self.h, chi, qref)

    def set_sponge_separable(self, chi_x=None, chi_y=None, chi_z=None, combine="max",
                             qref=None):
        lbm3_set_sponge_separable(self.h, chi_x, chi_y, chi_z, combine, qref)

    def step(self, n=1):
        lbm3_step(self.h, n)

    def sync(self):
        lbm3_sync(self.h)

    def populations(self):
        return lbm3_get_populations(self.h, self.shape)

    def set_populations(self, f):
        lbm3_set_populations(self.h, f)

    def moments(self):
        return lbm3_moments(self.h, self.shape)

    def steps_done(self):
        return lbm3_steps_done(self.h)

    def set_tuning(self, kernel=0, block=256):
        lbm3_set_tuning(self.h, kernel, block)

    def tuning(self):
        return lbm3_get_tuning(self.h)

    def autotune(self, reps=5):
        return lbm3_autotune(self.h, reps)

    def close(self):
        if self.h is not None:
            lbm3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
