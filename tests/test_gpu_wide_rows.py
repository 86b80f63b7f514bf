"""Rows wider than the strip kernels' byte offsets reach.

The K-step strip kernels address a lane's column within a row as a 32-bit
byte offset. An FP64 row of more than 2^29 cells is longer than that, so the
step must run such a lattice in the one-cell kernel whatever the tuning says,
and a batch (whose default launches are strips) must refuse it. The smallest
such lattice, 2^29 + 64 cells in one row, takes 77 GB for its two FP64
lattices, which one device holds."""
import pytest

from paper_1203_6350_amd import lbm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_fp64_rows_over_4gib_run_in_the_one_cell_kernel():
    import torch
    torch.cuda.set_device(0)
    lbm.load()
    # the lattices come from the library's own allocations: hand torch's
    # cached blocks back to the device first
    torch.cuda.empty_cache()
    nx, ny, steps = (1 << 29) + 64, 1, 5

    def run(tuning):
        say("case: wide FP64 row", nx, ny, tuning)
        g = torch.Generator(device="cuda").manual_seed(17)
        fields = [1.0 + 1e-3 * torch.randn(ny, nx, dtype=torch.float64, device="cuda", generator=g),
                  0.02 * torch.randn(ny, nx, dtype=torch.float64, device="cuda", generator=g),
                  0.02 * torch.randn(ny, nx, dtype=torch.float64, device="cuda", generator=g)]
        lat = lbm.Lattice(nx, ny, storage="f64", variant="II")
        try:
            lbm.lbm_init_fields_dev(lat.h, *fields)
            lat.set_tuning(**tuning)
            lat.step(steps)
            # the moments overwrite the fields, which the init has consumed
            lbm.lbm_moments_dev(lat.h, *fields)
            lat.sync()
            diag = lat.diagnostics()
            if tuning["kernel"] >= 2:
                with pytest.raises(lbm.LbmError) as e:
                    lbm.Batch([lat])
                assert e.value.code == lbm.LBM_EINVAL
        finally:
            lat.close()
        return fields, diag

    ref, ref_diag = run(dict(kernel=0, block=256, rows=0))
    got, got_diag = run(dict(kernel=4, block=64, rows=0))
    assert (got_diag == ref_diag).all()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    del ref, got
    torch.cuda.empty_cache()
