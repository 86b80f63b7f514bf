"""The D3Q15 step (Section 2 with the transform matrix of Appendix A.2) on the
GPU against the D3Q15 oracle.

Bars: FP64 storage, max |f_gpu - f_ref| <= 1e-12 max |f_ref|; FP32 storage,
relative L2 of p' = c_s^2 (rho - rho0) <= 1e-5; FP16 storage on smooth
acoustic fields, <= 1e-3. At the full 256^3 size of the bench workload the
oracle runs, per sampled cell, on the (2T+1)^3 box around it: after T steps a
cell depends only on cells within T in every axis, so the box centre is exact.
"""
import math

import numpy as np
import pytest

from oracle import d3q15 as o3
from paper_1203_6350_amd import lbm, workloads as wl

pytestmark = pytest.mark.gpu

S_MIX = (0.0, 0.0, 0.0, 0.0, 1.1, 1.2, 1.3, 1.4, 1.5, 1.6, 1.7, 1.8, 1.35, 1.45, 1.55)


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


def pprime_rel_l2(f_gpu, f_ref, rho0=1.0):
    rg = f_gpu.sum(axis=0) - rho0
    rr = f_ref.sum(axis=0) - rho0
    return math.sqrt(((rg - rr) ** 2).sum() / (rr ** 2).sum())


def noisy_fields(nx, ny, nz, seed, u0=(0.04, -0.01, 0.02), amp=1e-3):
    g = np.random.default_rng(seed)
    sh = (nz, ny, nx)
    rho = 1 + amp * g.standard_normal(sh)
    return (rho,) + tuple(u + amp * g.standard_normal(sh) for u in u0)


def profiles(nx, ny, nz, chi_max, width=None):
    return tuple(wl.quadratic_ramp_1d(n, width or max(1, n // 4), chi_max) for n in (nx, ny, nz))


def run3(fields, steps, *, sponge=None, qref=None, split=None, **cfg):
    """sponge: None, ("field", chi) or ("sep", (cx, cy, cz), combine)."""
    rho, ux, uy, uz = fields
    nz, ny, nx = rho.shape
    lat = lbm.Lattice3(nx, ny, nz, rho=rho, ux=ux, uy=uy, uz=uz, **cfg)
    if sponge is not None and sponge[0] == "field":
        lat.set_sponge(sponge[1], qref)
    elif sponge is not None:
        lat.set_sponge_separable(*sponge[1], combine=sponge[2], qref=qref)
    elif qref is not None:
        lat.set_sponge(None, qref)
    if split:
        lat.step(split)
        lat.step(steps - split)
    else:
        lat.step(steps)
    f = lat.populations()
    assert lat.steps_done() == steps
    lat.close()
    return f


QREF = (1.001, 0.05, -0.01, 0.015)
UB = dict(ux_base=0.04, uy_base=-0.01, uz_base=0.02)


# ------------------------------------------------------------------ FP64, every variant and sponge form

@pytest.mark.parametrize("variant", ["II", "I", "III", "none", "visc"])
@pytest.mark.parametrize("form", ["field", "max", "sum"])
def test_fp64_every_variant_and_sponge_form(variant, form):
    if variant == "visc" and form == "sum":
        pytest.skip("the viscosity ramp combines its profiles by max")
    nx, ny, nz, T = 37, 19, 11, 30
    say("case: D3Q15 FP64", variant, form)
    F = noisy_fields(nx, ny, nz, 11 + len(variant))
    chi_max = 1.0 if variant == "visc" else (0.1 if variant == "I" else 0.4)
    px, py, pz = profiles(nx, ny, nz, chi_max / (3 if form == "sum" else 1))
    chi = wl.sponge_3d(px, py, pz, "sum" if form == "sum" else "max")
    ref = o3.step(o3.feq_field(*F), T, s=S_MIX, chi=chi, qref=QREF, variant=variant)
    sponge = ("field", chi) if form == "field" else ("sep", (px, py, pz), form)
    got = run3(F, T, sponge=sponge, qref=QREF, split=13, storage="f64", variant=variant, s=S_MIX,
               **UB)
    e = rel_max(got, ref)
    say("  rel max %.3e" % e)
    assert e <= 1e-12


@pytest.mark.parametrize("nx,ny,nz", [(300, 5, 3), (1, 7, 5), (13, 1, 1), (1, 1, 1), (2, 3, 17)])
def test_fp64_ragged_and_degenerate_boxes(nx, ny, nz):
    """Rows longer than a block with a ragged tail, and boxes one cell thick
    (a pull along a one-cell axis reads the cell itself)."""
    T = 20
    say("case: D3Q15 FP64 box", nx, ny, nz)
    F = noisy_fields(nx, ny, nz, nx + 3 * ny + 7 * nz)
    chi = wl.sponge_3d(*profiles(nx, ny, nz, 0.3))
    ref = o3.step(o3.feq_field(*F), T, s=S_MIX, chi=chi, qref=QREF, variant="II", n=0.3, m=0.7)
    got = run3(F, T, sponge=("field", chi), qref=QREF, storage="f64", variant="II", s=S_MIX,
               shift_n=0.3, shift_m=0.7, **UB)
    assert rel_max(got, ref) <= 1e-12


def test_fp64_shift_parameters_and_rest_base():
    """n != m, base at rest while q_ref carries a mean flow."""
    nx, ny, nz, T = 24, 16, 12, 25
    F = noisy_fields(nx, ny, nz, 21, u0=(0.05, 0.0, 0.0))
    chi = wl.sponge_3d(*profiles(nx, ny, nz, 0.5))
    q = (1.0, 0.05, 0.0, 0.0)
    for var in ("II", "III"):
        ref = o3.step(o3.feq_field(*F), T, s=S_MIX, chi=chi, qref=q, variant=var, n=0.0, m=1.5)
        got = run3(F, T, sponge=("field", chi), qref=q, storage="f64", variant=var, s=S_MIX,
                   shift_n=0.0, shift_m=1.5)
        assert rel_max(got, ref) <= 1e-12, var


# ------------------------------------------------------------------ reduced precision

@pytest.mark.parametrize("storage,bar", [("f32", 1e-5), ("f16", 1e-3)])
@pytest.mark.parametrize("variant", ["II", "III"])
def test_reduced_precision_smooth_pulses(storage, bar, variant):
    """Mean flow Mach 0.17 along x, three pulses, a separable sponge of 12
    cells on every face; base = reference state (deviations O(1e-3))."""
    nx, ny, nz, T = 70, 45, 33, 60
    say("case: D3Q15", storage, variant)
    u0 = 0.1
    F = wl.gaussian_pulses_3d(nx, ny, nz, [(20, 20, 15), (45, 25, 18), (35, 12, 10)],
                              [1e-3, 6e-4, 8e-4], [4.0, 3.0, 5.0], 1.0, (u0, 0.0, 0.0))
    px, py, pz = profiles(nx, ny, nz, 0.3, width=12)
    q = (1.0, u0, 0.0, 0.0)
    ref = o3.step(o3.feq_field(*F), T, chi=wl.sponge_3d(px, py, pz), qref=q, variant=variant)
    got = run3(F, T, sponge=("sep", (px, py, pz), "max"), qref=q, storage=storage,
               variant=variant, ux_base=u0, f16_scale=5e-4)
    e = pprime_rel_l2(got, ref)
    say("  p' rel L2 %.3e" % e)
    assert e <= bar


def test_fp32_noise_every_variant():
    nx, ny, nz, T = 41, 23, 9, 30
    F = noisy_fields(nx, ny, nz, 31)
    for var in ("II", "I", "III", "none", "visc"):
        chi = wl.sponge_3d(*profiles(nx, ny, nz, 1.0 if var == "visc" else 0.3))
        ref = o3.step(o3.feq_field(*F), T, s=S_MIX, chi=chi, qref=QREF, variant=var)
        got = run3(F, T, sponge=("field", chi), qref=QREF, storage="f32", variant=var, s=S_MIX,
                   **UB)
        e = pprime_rel_l2(got, ref)
        say("  %s p' rel L2 %.3e" % (var, e))
        assert e <= 1e-5, var


# ------------------------------------------------------------------ sponge forms agree bitwise

@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_field_sponge_equals_separable_max_bitwise(storage):
    """max commutes with rounding to the compute type, so a full field equal
    to the separable max gives the same bits."""
    nx, ny, nz = 33, 20, 14
    F = noisy_fields(nx, ny, nz, 41, amp=2e-4)
    px, py, pz = profiles(nx, ny, nz, 0.35)
    kw = dict(storage=storage, variant="II", f16_scale=1e-3, **UB)
    a = run3(F, 15, sponge=("field", wl.sponge_3d(px, py, pz)), qref=QREF, **kw)
    b = run3(F, 15, sponge=("sep", (px, py, pz), "max"), qref=QREF, **kw)
    assert np.array_equal(a, b)


# ------------------------------------------------------------------ properties

def test_uniform_reference_state_is_a_fixed_point():
    """A uniform state equal to q_ref is left unchanged by every variant
    (the damping term vanishes and the equilibrium is the state)."""
    nx, ny, nz = 20, 12, 8
    q = (1.0, 0.06, -0.02, 0.03)
    F = tuple(np.full((nz, ny, nx), v) for v in q)
    chi = wl.sponge_3d(*profiles(nx, ny, nz, 0.4))
    f0 = o3.feq_field(*F)
    for var in ("II", "I", "III"):
        got = run3(F, 10, sponge=("field", chi), qref=q, storage="f64", variant=var)
        assert np.abs(got - f0).max() <= 1e-15, var


def test_mass_and_momentum_conserved_without_sponge():
    nx, ny, nz, T = 30, 26, 14, 50
    F = noisy_fields(nx, ny, nz, 51)
    f0 = o3.feq_field(*F)
    got = run3(F, T, storage="f64", variant="none", s=S_MIX, **UB)
    M, _Mi, cx, cy, cz, _w = o3.tables()
    for c in (np.ones(15), cx, cy, cz):
        a = np.tensordot(c, f0, axes=(0, 0)).sum()
        b = np.tensordot(c, got, axes=(0, 0)).sum()
        assert abs(a - b) <= 1e-12 * nx * ny * nz


def test_moments_match_oracle():
    nx, ny, nz, T = 26, 18, 10, 20
    F = noisy_fields(nx, ny, nz, 61)
    chi = wl.sponge_3d(*profiles(nx, ny, nz, 0.3))
    ref = o3.step(o3.feq_field(*F), T, s=S_MIX, chi=chi, qref=QREF, variant="II")
    lat = lbm.Lattice3(nx, ny, nz, rho=F[0], ux=F[1], uy=F[2], uz=F[3], storage="f64", s=S_MIX,
                       **UB)
    lat.set_sponge(chi, QREF)
    lat.step(T)
    got = lat.moments()
    lat.close()
    want = o3.moments(ref)
    for g, w in zip(got, want):
        assert np.abs(g - w).max() <= 1e-13


def test_set_get_populations_roundtrip_and_restart():
    """Populations written then read back; stepping from them matches the
    oracle from the same populations; the step count restarts at 0."""
    nx, ny, nz = 21, 13, 7
    F = noisy_fields(nx, ny, nz, 71)
    f = o3.feq_field(*F) + 1e-5 * np.random.default_rng(2).standard_normal((15, nz, ny, nx))
    lat = lbm.Lattice3(nx, ny, nz, storage="f64", s=S_MIX, **UB)
    lat.step(3)
    lat.set_populations(f)
    assert lat.steps_done() == 0
    assert np.abs(lat.populations() - f).max() <= 1e-15
    lat.step(9)
    got = lat.populations()
    lat.close()
    ref = o3.step(f, 9, s=S_MIX, variant="II")
    assert rel_max(got, ref) <= 1e-12


def test_bad_sponge_arguments_rejected():
    lat = lbm.Lattice3(6, 5, 4, storage="f32", variant="visc")
    bad = np.zeros((4, 5, 6))
    bad[1, 2, 3] = 1.5
    with pytest.raises(lbm.LbmError):
        lat.set_sponge(bad)
    with pytest.raises(lbm.LbmError):
        lat.set_sponge_separable(np.zeros(6), None, None, combine="sum")
    with pytest.raises(lbm.LbmError):
        lat.set_sponge(None, (0.0, 0.0, 0.0, 0.0))
    with pytest.raises(lbm.LbmError):
        lat.step(-1)
    lat.close()
    lat = lbm.Lattice3(6, 5, 4, storage="f32", variant="II")
    bad[1, 2, 3] = -0.1
    with pytest.raises(lbm.LbmError):
        lat.set_sponge(bad)
    lat.close()


# ------------------------------------------------------------------ full size, sampled

@pytest.mark.parametrize("storage,bar", [("f32", 1e-5), ("f16", 1e-3)])
def test_full_size_cube_sampled_against_oracle(storage, bar):
    """256^3 Type II with mean flow, 16 pulses and the six-face ramp (the
    bench workload, in the launch shape the bench times: one cell per thread
    in FP32, two in FP16), T = 12 steps; 24 sampled cells (pulse centres,
    sponge, random) against the oracle on the 25^3 box around each."""
    spec = wl.cube_d3q15()
    n, T = spec["n"], 12
    say("case: D3Q15 256^3 sampled", storage)
    F = spec["fields"]()
    prof = spec["profile"]
    lat = lbm.Lattice3(n, n, n, rho=F[0], ux=F[1], uy=F[2], uz=F[3], storage=storage,
                       variant="II", ux_base=spec["u0"], f16_scale=1e-3)
    assert lat.tuning()["kernel"] == (1 if storage == "f16" else 0)
    lat.set_sponge_separable(prof, prof, prof, "max", spec["qref"])
    lat.step(T)
    rho_g = lat.moments()[0]
    lat.close()
    g = np.random.default_rng(9)
    top = np.argsort(np.abs(F[0] - 1.0).ravel())[-8:]
    samples = [np.unravel_index(i, F[0].shape) for i in top]
    samples += [(int(a), int(b), int(c)) for a, b, c in g.integers(0, 20, (8, 3))]
    samples += [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(8)]
    amp = np.abs(rho_g - 1.0).max()
    worst = 0.0
    for (z, y, x) in samples:
        idx = [np.arange(c - T, c + T + 1) % n for c in (z, y, x)]
        sub = [a[np.ix_(*idx)] for a in F]
        chi = wl.sponge_3d(prof[idx[2]], prof[idx[1]], prof[idx[0]])
        ref = o3.step(o3.feq_field(*sub), T, chi=chi, qref=spec["qref"], variant="II")
        rho_r = ref[:, T, T, T].sum()
        worst = max(worst, abs(rho_g[z, y, x] - rho_r) / amp)
    say("  worst sampled |d rho| / max |rho'| = %.3e" % worst)
    assert worst <= bar


# ------------------------------------------------------------------ launch shapes

@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("nx,ny,nz", [(16, 5, 3), (40, 9, 7), (8, 1, 2), (600, 3, 2), (21, 4, 3), (2, 3, 2),
                                      (1, 4, 3), (1, 1, 1)])
def test_every_launch_shape_bitwise_identical(storage, nx, ny, nz):
    """One and two cells per thread with every workgroup size: the same bits
    (rows shorter and longer than a workgroup, ragged tails, the periodic
    wrap at row ends); FP64 against the oracle."""
    say("case: D3Q15 shapes", storage, nx, ny, nz)
    F = noisy_fields(nx, ny, nz, 81 + nx)
    chi = wl.sponge_3d(*profiles(nx, ny, nz, 0.3))
    shapes = [(0, b) for b in (64, 128, 256, 320, 512)]
    shapes += [(1, b) for b in (64, 256, 512) if nx % 2 == 0]
    states = []
    for k, b in shapes:
        lat = lbm.Lattice3(nx, ny, nz, rho=F[0], ux=F[1], uy=F[2], uz=F[3], storage=storage,
                           variant="II", s=S_MIX, f16_scale=1e-3, **UB)
        lat.set_sponge(chi, QREF)
        lat.set_tuning(kernel=k, block=b)
        assert lat.tuning() == {"kernel": k, "block": b}
        lat.step(7)
        states.append(((k, b), lat.populations()))
        lat.close()
    for t, st in states[1:]:
        assert np.array_equal(st, states[0][1]), t
    if storage == "f64":
        ref = o3.step(o3.feq_field(*F), 7, s=S_MIX, chi=chi, qref=QREF, variant="II")
        assert rel_max(states[-1][1], ref) <= 1e-12


def test_bad_launch_shape_rejected():
    lat = lbm.Lattice3(13, 4, 4, storage="f16")
    assert lat.tuning() == {"kernel": 0, "block": 256}     # odd nx
    for k, b in ((0, 0), (0, 32), (0, 96), (0, 1024), (2, 256), (1, 256)):
        with pytest.raises(lbm.LbmError):
            lat.set_tuning(kernel=k, block=b)
    lat.close()
    lat = lbm.Lattice3(12, 4, 4, storage="f16")
    assert lat.tuning() == {"kernel": 1, "block": 256}
    lat.close()
    lat = lbm.Lattice3(12, 4, 4, storage="f32")
    assert lat.tuning() == {"kernel": 0, "block": 256}
    lat.set_tuning(kernel=1, block=128)
    lat.close()


def test_autotune_keeps_state():
    nx, ny, nz = 48, 20, 12
    F = noisy_fields(nx, ny, nz, 95)
    lat = lbm.Lattice3(nx, ny, nz, rho=F[0], ux=F[1], uy=F[2], uz=F[3], storage="f32", **UB)
    lat.set_sponge(wl.sponge_3d(*profiles(nx, ny, nz, 0.3)), QREF)
    lat.step(3)
    before = lat.populations()
    best, ms = lat.autotune(reps=2)
    assert ms > 0 and best == lat.tuning() and best["kernel"] in (0, 1)
    assert np.array_equal(lat.populations(), before)
    assert lat.steps_done() == 3
    lat.close()
