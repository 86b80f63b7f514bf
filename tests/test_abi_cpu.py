"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the headers under include/ declare, and rejects bad arguments
before it touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1203_6350_amd import lbm, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def declared_functions():
    names = []
    for header in HEADERS:
        src = open(header).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(\w+)\s*\(", src,
                            flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "lbm_create" in names and "vn_amplification" in names and len(names) >= 18
    assert "lbm3_create" in names and "lbm3_step" in names
    L = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    L = lbm.load()
    for n in declared_functions():
        assert hasattr(L, n)
        if n not in ("lbm_destroy", "lbm_last_error", "lbm_batch_destroy", "lbm3_destroy"):
            assert getattr(L, n).argtypes is not None, n


def test_struct_layouts_match_header():
    assert ctypes.sizeof(lbm.lbm_config) == 8 * 2 + 8 * 3 + 8 * 9 + 8 * 2 + 4 * 2 + 8 + 8
    assert ctypes.sizeof(lbm.lbm_vn_params) == 8 * 9 + 8 * 6 + 4 * 2
    assert ctypes.sizeof(lbm.lbm_qref) == 24
    assert ctypes.sizeof(lbm.lbm3_config) == 8 * 3 + 8 * 4 + 8 * 15 + 8 * 2 + 4 * 2 + 8 + 8
    assert ctypes.sizeof(lbm.lbm3_qref) == 32


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(nz=-1), dict(rho_base=0.0), dict(uz_base=float("inf")),
    dict(s=(0,) * 4 + (2.5,) + (1.9,) * 10), dict(storage=7), dict(variant=9),
    dict(storage="f16", f16_scale=0.0), dict(shift_m=-0.5), dict(nx=2048, ny=2048, nz=1024),
])
def test_create3_rejects_bad_config(bad):
    kw = dict(nx=4, ny=4, nz=4)
    kw.update(bad)
    nx, ny, nz = kw.pop("nx"), kw.pop("ny"), kw.pop("nz")
    cfg = lbm.make_config3(nx, ny, nz, **kw)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm3_create(cfg)
    assert e.value.code == lbm.LBM_EINVAL
    assert lbm.lbm_last_error()


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(rho_base=0.0), dict(rho_base=float("nan")),
    dict(s=(0, 0, 0, 2.5, 1.9, 1.9, 1.9, 1.9, 1.9)), dict(storage=7), dict(variant=9),
    dict(storage="f16", f16_scale=0.0), dict(shift_n=-0.5), dict(nx=70000, ny=70000),
])
def test_create_rejects_bad_config(bad):
    kw = dict(nx=8, ny=8)
    kw.update(bad)
    nx, ny = kw.pop("nx"), kw.pop("ny")
    cfg = lbm.make_config(nx, ny, **kw)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(cfg)
    assert e.value.code == lbm.LBM_EINVAL
    assert lbm.lbm_last_error()


@pytest.mark.parametrize("nx,ny,ok", [
    (46340, 46340, True), (46341, 46341, False),      # nx * ny below 2^31
    (1 << 30, 1, True), ((1 << 30) + 1, 1, False),    # one side at most 2^30
    (1, 1 << 30, True), (2, 1 << 30, False),
])
def test_size_limit_is_exact(nx, ny, ok):
    """The largest lattices the library takes (nx * ny below 2^31, each side
    at most 2^30) are accepted (sized on the host, nothing allocated) and
    the next ones are rejected."""
    cfg = lbm.make_config(nx, ny, storage="f16", f16_scale=1e-3)
    if ok:
        plane = -(-nx * ny * 2 // 256) * 256
        assert lbm.lbm_required_bytes(cfg) == 2 * 9 * plane
    else:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_required_bytes(cfg)
        assert e.value.code == lbm.LBM_EINVAL


def test_required_bytes_is_host_only():
    cfg = lbm.make_config(100, 30, storage="f32")
    b = lbm.lbm_required_bytes(cfg)
    # two lattices, nine planes, planes rounded to 256 bytes
    plane = -(-100 * 30 * 4 // 256) * 256
    assert b == 2 * 9 * plane


def test_null_handle_calls_fail_cleanly():
    L = lbm.load()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_sync(None) == lbm.LBM_EINVAL
    L.lbm_destroy(None)  # accepted
    out = np.empty(7)
    assert L.lbm_diagnostics(None, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lbm.LBM_EINVAL


def test_vn_rejects_bad_parameters():
    bad = dict(s=(1.9,) * 9, chi=-1.0, qref=(1, 0, 0), variant="II")
    with pytest.raises(lbm.LbmError) as e:
        lbm.vn_amplification(bad, np.zeros(4), np.zeros(4))
    assert e.value.code == lbm.LBM_EINVAL


def test_sponge_generators():
    """Workload generators: the quadratic ramp is chi_max at the edge cell and
    zero from depth W; the normalised sigma~ of eq. normalizedsigma peaks at 1
    at 4/5 of the layer and vanishes at both layer ends (Section 2.3)."""
    r = wl.quadratic_ramp_1d(64, 10, 0.2)
    assert r[0] == r[-1] == pytest.approx(0.2)
    assert np.all(r[10:54] == 0)
    assert np.all(np.diff(r[:11]) < 0)
    W = 1000
    s = wl.orszag_profile_1d(2 * W + 10, W, 1.0)
    xi = wl.ramp_depth(2 * W + 10, W)
    i = np.argmax(s[:W + 1])
    assert s[i] == pytest.approx(1.0, abs=1e-5)
    assert xi[i] == pytest.approx(0.8, abs=2e-3)
    assert s[W] == 0.0
    two = wl.sponge_2d(r, r)
    assert two.shape == (64, 64) and two[0, 30] == pytest.approx(0.2) and two[30, 30] == 0


@pytest.mark.parametrize("every_n,max_dev,msg", [
    (-1, 1.0, "every_n"), (10, 0.0, "max_dev"), (10, -1.0, "max_dev"),
    (10, float("nan"), "max_dev"), (10, 1.0, "handle"), (0, float("nan"), "handle"),
])
def test_detector_rejects_bad_arguments(every_n, max_dev, msg):
    """lbm_set_detector checks its arguments before the handle: a negative
    period or a max_dev that is not > 0 (NaN included) is EINVAL; with good
    arguments a NULL handle is EINVAL; every_n = 0 (off) ignores max_dev."""
    L = lbm.load()
    assert L.lbm_set_detector(None, every_n, max_dev) == lbm.LBM_EINVAL
    assert msg in lbm.lbm_last_error()


def test_detector_status_null_arguments():
    L = lbm.load()
    t = ctypes.c_int64(0)
    assert L.lbm_detector_status(None, ctypes.byref(t)) == lbm.LBM_EINVAL
    assert L.lbm_batch_detector_status(None, ctypes.byref(t)) == lbm.LBM_EINVAL
    assert L.lbm_batch_sync(None) == lbm.LBM_EINVAL


def test_unstable_error_carries_the_result():
    """The binding raises LbmUnstable (an LbmError) for LBM_EUNSTABLE and
    keeps the outputs the call wrote."""
    with pytest.raises(lbm.LbmError) as e:
        lbm._check(lbm.LBM_EUNSTABLE, result=np.arange(7.0))
    assert isinstance(e.value, lbm.LbmUnstable) and e.value.code == lbm.LBM_EUNSTABLE
    np.testing.assert_array_equal(e.value.result, np.arange(7.0))


def test_device_sponge_rejects_bad_arguments():
    L = lbm.load()
    q = lbm.lbm_qref(1.0, 0.0, 0.0)
    assert L.lbm_set_sponge_separable_dev(None, None, None, 0, None) == lbm.LBM_EINVAL
    assert "handle" in lbm.lbm_last_error()
