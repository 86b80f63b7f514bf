"""The acoustic line source with outflow (Sec. 4.2) on the GPU against the
oracle's channel stepper."""
import math

import numpy as np
import pytest

import oracle
from paper_1203_6350_amd import lbm, workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    lbm.load()
    yield


def rel_max(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


SRC = (1.0, 2e-4, 0.01, 0.7, 0.05, 0.0)


@pytest.mark.parametrize("variant", ["II", "I", "III", "none", "visc"])
@pytest.mark.parametrize("outflow", [True, False])
def test_channel_fp64_against_oracle(variant, outflow):
    """FP64 populations within 1e-12 of max |f| after 150 steps on a ragged
    channel (131 x 23), 2-D sponge before the outflow, steps split over
    several calls (the source phase follows the handle's step count)."""
    nx, ny, T = 131, 23, 150
    say("case: channel FP64", variant, outflow)
    g = np.random.default_rng(5)
    rho = 1 + 1e-4 * g.standard_normal((ny, nx))
    ux = 0.05 + 1e-4 * g.standard_normal((ny, nx))
    uy = 1e-4 * g.standard_normal((ny, nx))
    ramp = wl.quadratic_ramp_1d(nx, 30, 0.1 if variant == "I" else 0.4)
    chi = np.tile(np.where(np.arange(nx) > nx // 2, ramp, 0.0), (ny, 1))
    f0 = oracle.feq_field(rho, ux, uy)
    ref = oracle.step_line_source(f0, T, source=SRC, outflow=outflow, chi=chi, variant=variant,
                                  qref=(1.0, 0.05, 0.0))
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f64", variant=variant, ux_base=0.05)
    lat.set_sponge(chi, (1.0, 0.05, 0.0))
    lat.set_line_source(SRC, outflow)
    lat.step(61)
    lat.step(T - 61)
    got = lat.populations()
    lat.close()
    assert rel_max(got, ref) <= 1e-12


@pytest.mark.parametrize("storage,bar", [("f32", 1e-5), ("f16", 2e-3)])
def test_channel_reduced_precision(storage, bar):
    """The emitted wave in FP32/FP16 storage: p' against the FP64 oracle,
    relative L2 over the channel (equilibrium base at the mean flow)."""
    nx, ny, T = 400, 8, 600
    rho = np.ones((ny, nx))
    ux = np.full((ny, nx), 0.05)
    uy = np.zeros((ny, nx))
    chi = np.tile(wl.quadratic_ramp_1d(nx, 80, 0.5) * (np.arange(nx) > 200), (ny, 1))
    f0 = oracle.feq_field(rho, ux, uy)
    ref = oracle.step_line_source(f0, T, source=SRC, chi=chi, variant="II", qref=(1.0, 0.05, 0.0))
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage=storage, variant="II", ux_base=0.05,
                      f16_scale=2e-4)
    lat.set_sponge(chi, (1.0, 0.05, 0.0))
    lat.set_line_source(SRC)
    lat.step(T)
    got = lat.populations()
    lat.close()
    rg, rr = got.sum(axis=0) - 1.0, ref.sum(axis=0) - 1.0
    e = math.sqrt(((rg - rr) ** 2).sum() / (rr ** 2).sum())
    say("  %s channel p' rel L2 %.3e" % (storage, e))
    assert e <= bar


def test_channel_checks_and_reset():
    lat = lbm.Lattice(2, 4, storage="f64")
    with pytest.raises(lbm.LbmError):
        lat.set_line_source(SRC)          # nx < 3
    lat.close()
    nx, ny = 30, 6
    lat = lbm.Lattice(nx, ny, storage="f32", variant="II")
    with pytest.raises(lbm.LbmError):
        lat.set_line_source((1.0, 1.5, 0.01, 0.0, 0.0, 0.0))   # density would turn negative
    lat.set_line_source(SRC)
    with pytest.raises(lbm.LbmError):
        lbm.Batch([lat])
    with pytest.raises(lbm.LbmError):
        lat.set_qref_field(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    lat.set_line_source(None)
    lat.step(3)
    b = lbm.Batch([lat])                  # periodic again: batchable
    b.close()
    lat.close()


def test_paper_line_source_full_size_against_one_row_oracle():
    """The paper's line-source channel at its size (800 x 200, Type II layer of
    0.8, Re = 1e6, mean flow 0.1, sampled at T_m + 10 T_p = 2182 steps): every
    GPU row is bit-identical and equals the one-row FP64 oracle (the set-up is
    y-invariant) within 1e-12 of max |f|."""
    cfg = wl.paper_line_source("II", u0=0.1)
    nx, ny, T, u0 = cfg["nx"], cfg["ny"], cfg["t_sample"], cfg["u0"]
    say("case: paper line source", nx, ny, T)
    f0 = oracle.feq_field(np.ones((1, nx)), np.full((1, nx), u0), np.zeros((1, nx)))
    ref = oracle.step_line_source(f0, T, source=cfg["source"], s=cfg["s"],
                                  chi=cfg["profile"][None, :], variant="II", qref=(1.0, u0, 0.0))
    lat = lbm.Lattice(nx, ny, rho=np.ones((ny, nx)), ux=np.full((ny, nx), u0),
                      uy=np.zeros((ny, nx)), storage="f64", variant="II", s=cfg["s"], ux_base=u0)
    lat.set_sponge_separable(cfg["profile"], None, "max", (1.0, u0, 0.0))
    lat.set_line_source(cfg["source"])
    lat.step(T)
    f = lat.populations()
    lat.close()
    assert (f == f[:, :1, :]).all()
    assert rel_max(f[:, :1, :], ref) <= 1e-12
