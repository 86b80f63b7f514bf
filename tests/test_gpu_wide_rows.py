"""Rows at the limit of the strip kernels' 32-bit row addressing.

The K-step strip kernels address a lane's column within a row as a 32-bit
byte offset and read a row through a buffer range of the row's byte count,
also 32 bits. An FP64 row of 2^29 cells or more (2^32 bytes or more) is
beyond that, so the step must run such a lattice in the one-cell kernel
whatever the tuning says, and a batch (whose default launches are strips)
must refuse it; a row just below the limit runs in the strips, whose last
cells sit at the top of the 32-bit range. Both are checked bit for bit
against the one-cell kernel. Each lattice pair takes about 77 GB, which one
device holds; the runs follow one another."""
import pytest

from paper_1203_6350_amd import lbm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("nx,strips", [((1 << 29) - 64, True), (1 << 29, False)])
def test_fp64_rows_at_the_32_bit_limit(nx, strips):
    import torch
    torch.cuda.set_device(0)
    lbm.load()
    # the lattices come from the library's own allocations: hand torch's
    # cached blocks back to the device first
    torch.cuda.empty_cache()
    ny, steps = 1, 5

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
                # batches take exactly the rows the strips take
                if strips:
                    lbm.Batch([lat]).close()
                else:
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
