"""GPU test of lbm_diagnostics_dev_noalloc (the allocation-free variant of
lbm_diagnostics_dev, partials in a static device array): through the C ABI,
on two calls in a row (the second on a smaller lattice, so stale partials of
the first would show), its output equals lbm_diagnostics_dev's bit for bit
in every storage mode."""
import ctypes

import numpy as np
import pytest

from paper_1203_6350_amd import lbm, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    lbm.load()
    yield


def make(nx, ny, storage, steps):
    rho, ux, uy = wl.gaussian_pulses(nx, ny, [((nx - 1) / 2, (ny - 1) / 2)], [1e-3], [6.0],
                                     u0=(0.05, 0.0))
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage=storage, variant="II",
                      ux_base=0.05, f16_scale=1e-3)
    prof = wl.quadratic_ramp_1d(nx, max(1, nx // 8), 0.3)
    lat.set_sponge_separable(prof, None, "max", (1.0, 0.05, 0.0))
    lat.step(steps)
    return lat


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_noalloc_diagnostics_equal_allocating_ones(storage):
    import torch
    L = lbm.load()
    print("case: noalloc diagnostics", storage, flush=True)
    for nx, ny, steps in ((1500, 900, 13), (37, 11, 5)):
        lat = make(nx, ny, storage, steps)
        a = torch.full((7,), -1.0, dtype=torch.float64, device="cuda")
        b = torch.full((7,), -2.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        assert L.lbm_diagnostics_dev_noalloc(lat.h, ctypes.c_void_p(a.data_ptr())) == lbm.LBM_OK
        assert L.lbm_diagnostics_dev(lat.h, ctypes.c_void_p(b.data_ptr())) == lbm.LBM_OK
        lat.sync()
        torch.cuda.synchronize()
        ga, gb = a.cpu().numpy(), b.cpu().numpy()
        print(nx, ny, ga, flush=True)
        np.testing.assert_array_equal(ga, gb)
        np.testing.assert_array_equal(ga, lat.diagnostics())
        assert ga[6] == 0 and ga[5] > 0
        lat.close()


def test_noalloc_rejects_null_arguments():
    L = lbm.load()
    assert L.lbm_diagnostics_dev_noalloc(None, None) == lbm.LBM_EINVAL
