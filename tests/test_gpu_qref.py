"""Per-cell and time-averaged reference state on the GPU against the oracle
(the paper's q_ref as a function of space and time: Sec. 1, Sec. 2.2)."""
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


def case(nx, ny, seed, u0=0.04):
    g = np.random.default_rng(seed)
    rho = 1 + 1e-3 * g.standard_normal((ny, nx))
    ux = u0 + 1e-3 * g.standard_normal((ny, nx))
    uy = 1e-3 * g.standard_normal((ny, nx))
    chi = g.uniform(0, 0.4, (ny, nx)) * (g.uniform(size=(ny, nx)) < 0.6)
    rf = 1 + 5e-4 * g.standard_normal((ny, nx))
    uxf = u0 + 5e-4 * g.standard_normal((ny, nx))
    uyf = 5e-4 * g.standard_normal((ny, nx))
    return rho, ux, uy, chi, (rf, uxf, uyf)


def rel_max(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def conserved(q):
    rf, uxf, uyf = q
    return np.stack([rf, rf * uxf, rf * uyf])


@pytest.mark.parametrize("variant", ["I", "II", "III", "none", "visc"])
@pytest.mark.parametrize("alpha", [0.0, 0.02, 1.0])
def test_reference_field_fp64_against_oracle(variant, alpha):
    """FP64: populations within 1e-12 of max |f| and the reference field
    within 1e-12 of the oracle after 30 steps (ragged 77 x 45, 2-D sponge)."""
    nx, ny, T = 77, 45, 30
    say("case: reference field FP64", variant, alpha)
    rho, ux, uy, chi, q = case(nx, ny, 3 + len(variant))
    if variant == "I":
        chi = np.minimum(chi, 0.1)
    if variant == "visc":
        chi = np.minimum(chi, 1.0)
    f0 = oracle.feq_field(rho, ux, uy)
    ref, cf = oracle.step_avg(f0, conserved(q), T, alpha=alpha, chi=chi, variant=variant)
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f64", variant=variant, ux_base=0.04)
    lat.set_sponge(chi, (1.0, 0.04, 0.0))
    lat.set_qref_field(*q)
    if alpha:
        lat.set_qref_average(alpha)
    lat.step(T)
    got = lat.populations()
    rf, uxf, uyf = lat.qref_field()
    lat.close()
    assert rel_max(got, ref) <= 1e-12
    np.testing.assert_allclose(rf, cf[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rf * uxf, cf[1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rf * uyf, cf[2], rtol=0, atol=1e-12)


@pytest.mark.parametrize("form", ["max", "sum", "zero"])
def test_reference_field_with_separable_sponge_fp64(form):
    nx, ny, T = 64, 50, 25
    rho, ux, uy, chi, q = case(nx, ny, 17)
    g = np.random.default_rng(18)
    cx = g.uniform(0, 0.2, nx)
    cy = g.uniform(0, 0.2, ny)
    chi2 = (np.maximum(cy[:, None], cx[None, :]) if form == "max" else
            cy[:, None] + cx[None, :] if form == "sum" else np.zeros((ny, nx)))
    f0 = oracle.feq_field(rho, ux, uy)
    ref, _ = oracle.step_avg(f0, conserved(q), T, alpha=0.1, chi=chi2, variant="II")
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f64", variant="II", ux_base=0.04)
    if form == "zero":
        lat.set_sponge(None, (1.0, 0.04, 0.0))
    else:
        lat.set_sponge_separable(cx, cy, form, (1.0, 0.04, 0.0))
    lat.set_qref_field(*q)
    lat.set_qref_average(0.1)
    lat.step(T)
    got = lat.populations()
    lat.close()
    assert rel_max(got, ref) <= 1e-12


@pytest.mark.parametrize("storage,bar", [("f32", 1e-5), ("f16", 1e-3)])
def test_reference_field_reduced_precision(storage, bar):
    """Reduced-precision storage with an averaged reference: the pressure
    fluctuation p' = c_s^2 (rho - rho0) against the FP64 oracle, relative to
    the initial fluctuation (rounding noise does not shrink with the damped
    signal)."""
    n, T = 96, 200
    rho, ux, uy = wl.gaussian_pulses(n, n, [(48, 48)], [1e-3], [6.0], u0=(0.05, 0.0))
    chi = wl.sponge_2d(wl.quadratic_ramp_1d(n, 16, 0.2), wl.quadratic_ramp_1d(n, 16, 0.2))
    q = (np.ones((n, n)), np.full((n, n), 0.05), np.zeros((n, n)))
    f0 = oracle.feq_field(rho, ux, uy)
    ref, _ = oracle.step_avg(f0, conserved(q), T, alpha=0.01, chi=chi, variant="II")
    lat = lbm.Lattice(n, n, rho=rho, ux=ux, uy=uy, storage=storage, variant="II", ux_base=0.05,
                      f16_scale=1e-3)
    lat.set_sponge(chi, (1.0, 0.05, 0.0))
    lat.set_qref_field(*q)
    lat.set_qref_average(0.01)
    lat.step(T)
    got = lat.populations()
    lat.close()
    rg = got.sum(axis=0) - 1.0
    rr = ref.sum(axis=0) - 1.0
    r0 = f0.sum(axis=0) - 1.0
    e = math.sqrt(((rg - rr) ** 2).sum() / (r0 ** 2).sum())
    say("  %s p' error / initial %.3e" % (storage, e))
    assert e <= bar


def test_uniform_field_equals_uniform_reference_bitwise():
    """A field equal everywhere to the uniform q_ref (fixed, alpha = 0) gives
    the same bits as the uniform reference in the one-cell kernel; clearing
    the field returns to the uniform path."""
    nx, ny = 90, 33
    rho, ux, uy, chi, _ = case(nx, ny, 31)
    qu = (1.0003, 0.041, -0.002)
    outs = []
    for mode in ("uniform", "field", "cleared"):
        lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f32", variant="II", ux_base=0.04)
        lat.set_tuning(kernel=0, block=256)
        lat.set_sponge(chi, qu)
        if mode != "uniform":
            lat.set_qref_field(np.full((ny, nx), qu[0]), np.full((ny, nx), qu[1]),
                               np.full((ny, nx), qu[2]))
        if mode == "cleared":
            lat.step(3)
            lat.set_qref_field(None, None, None)
        lat.step(20 if mode != "cleared" else 17)
        outs.append(lat.save_state())
        lat.close()
    np.testing.assert_array_equal(outs[1], outs[0])
    np.testing.assert_array_equal(outs[2], outs[0])


def test_reference_field_round_trip_and_batch_refusal():
    nx, ny = 40, 30
    rho, ux, uy, chi, q = case(nx, ny, 41)
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f64", variant="II", ux_base=0.04)
    lat.set_qref_field(*q)
    for a, b in zip(lat.qref_field(), q):
        np.testing.assert_allclose(a, b, rtol=1e-15, atol=1e-15)
    lbm.Batch([lat]).close()  # a fixed field is batched, a running mean is not
    lat.set_qref_average(0.25)
    with pytest.raises(lbm.LbmError):
        lbm.Batch([lat])
    lat.set_qref_average(0.0)
    with pytest.raises(lbm.LbmError):
        lat.set_qref_average(1.5)
    lat.set_qref_field(None, None, None)
    with pytest.raises(lbm.LbmError):
        lat.set_qref_average(0.1)
    lat.close()


STRIP_TUNINGS = [dict(kernel=2, block=128, rows=5), dict(kernel=3, block=256, rows=0),
                 dict(kernel=4, block=64, rows=7), dict(kernel=4, block=128, rows=0)]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("variant", ["II", "I", "III", "none", "visc"])
def test_fixed_reference_field_in_strip_kernels_bitwise(storage, variant):
    """A per-cell reference state fixed in time runs in the multi-step strip
    kernels (the row's field values travel with its sponge input): every
    strip shape gives the bits of the one-cell-per-thread kernel, for every
    sponge form, with whole launches and a remainder (11 steps); FP64 against
    the oracle."""
    nx, ny, T = 133, 37, 11
    say("case: fixed reference field in strips", storage, variant)
    rho, ux, uy, chi, q = case(nx, ny, 40 + len(variant))
    if variant == "I":
        chi = np.minimum(chi, 0.1)
    if variant == "visc":
        chi = np.minimum(chi, 1.0)
    g = np.random.default_rng(9)
    cx = np.minimum(g.uniform(0, 0.3, nx) * (g.uniform(size=nx) < 0.4), chi.max())
    cy = np.minimum(g.uniform(0, 0.3, ny) * (g.uniform(size=ny) < 0.4), chi.max())
    for form in ("field", "max", "sum"):
        states = []
        for t in [dict(kernel=0, block=256)] + STRIP_TUNINGS:
            lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage=storage, variant=variant,
                              ux_base=0.04, f16_scale=1e-3)
            if form == "field":
                lat.set_sponge(chi, (1.0, 0.04, 0.0))
            else:
                lat.set_sponge_separable(cx, cy, form, (1.0, 0.04, 0.0))
            lat.set_qref_field(*q)
            lat.set_tuning(**t)
            lat.step(T)
            states.append(lat.save_state())
            if storage == "f64" and form == "field" and t == STRIP_TUNINGS[-1]:
                got = lat.populations()
            lat.close()
        for t, st in zip(STRIP_TUNINGS, states[1:]):
            assert (st == states[0]).all(), (form, t)
    if storage == "f64":
        ref, _ = oracle.step_avg(oracle.feq_field(rho, ux, uy), conserved(q), T, alpha=0.0,
                                 chi=chi, variant=variant)
        assert rel_max(got, ref) <= 1e-12


def test_reference_field_other_parameters_use_one_step_kernel():
    """Rates or shifts other than the default form, and a running mean,
    keep the reference field in the one-cell kernel: still the oracle's
    result (FP64) under a strip tuning."""
    nx, ny, T = 70, 33, 9
    rho, ux, uy, chi, q = case(nx, ny, 61)
    S = (0.0, 0.3, 0.0, 1.2, 1.3, 1.4, 1.5, 1.6, 1.7)
    for kw, alpha in ((dict(s=S), 0.0), (dict(shift_n=0.3, shift_m=0.7), 0.0), ({}, 0.05)):
        lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f64", variant="II",
                          ux_base=0.04, **kw)
        lat.set_sponge(chi, (1.0, 0.04, 0.0))
        lat.set_qref_field(*q)
        if alpha:
            lat.set_qref_average(alpha)
        lat.set_tuning(kernel=4, block=128, rows=0)
        lat.step(T)
        got = lat.populations()
        lat.close()
        ref, _ = oracle.step_avg(oracle.feq_field(rho, ux, uy), conserved(q), T, alpha=alpha,
                                 chi=chi, variant="II", s=kw.get("s", oracle.S_MRT_DEFAULT),
                                 n=kw.get("shift_n", 0.5), m=kw.get("shift_m", 0.5))
        assert rel_max(got, ref) <= 1e-12, kw


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("variant", ["II", "I", "III", "none", "visc"])
@pytest.mark.parametrize("nx,ny", [(101, 31), (1, 7), (66, 1)])
def test_running_mean_reference_in_strip_kernels_bitwise(storage, variant, nx, ny):
    """The running-mean reference in the strip kernels (each launch reads the
    field and writes the updated one to a second buffer): populations and
    field bit-identical to the one-cell kernel's in-place update for every
    strip shape and sponge form, over whole launches and a remainder, and
    across a later change of alpha, also on a single column and a single
    row; FP64 against the oracle."""
    say("case: running-mean reference in strips", storage, variant, nx, ny)
    rho, ux, uy, chi, q = case(nx, ny, 70 + len(variant))
    if variant == "I":
        chi = np.minimum(chi, 0.1)
    if variant == "visc":
        chi = np.minimum(chi, 1.0)
    g = np.random.default_rng(19)
    cx = np.minimum(g.uniform(0, 0.3, nx) * (g.uniform(size=nx) < 0.4), chi.max() / 2)
    cy = np.minimum(g.uniform(0, 0.3, ny) * (g.uniform(size=ny) < 0.4), chi.max() / 2)
    for form in ("field", "sum"):
        results = []
        for t in [dict(kernel=0, block=256)] + STRIP_TUNINGS:
            lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage=storage, variant=variant,
                              ux_base=0.04, f16_scale=1e-3)
            if form == "field":
                lat.set_sponge(chi, (1.0, 0.04, 0.0))
            else:
                lat.set_sponge_separable(cx, cy, form, (1.0, 0.04, 0.0))
            lat.set_qref_field(*q)
            lat.set_tuning(**t)
            lat.set_qref_average(0.03)
            lat.step(9)
            lat.set_qref_average(0.5)
            lat.step(6)
            results.append((lat.save_state(), np.stack(lat.qref_field())))
            if storage == "f64" and form == "field" and t == STRIP_TUNINGS[-1]:
                got = lat.populations()
            lat.close()
        for t, (st, qf) in zip(STRIP_TUNINGS, results[1:]):
            assert (st == results[0][0]).all(), (form, t)
            assert np.array_equal(qf, results[0][1]), (form, t)
    if storage == "f64":
        f0 = oracle.feq_field(rho, ux, uy)
        ref, cf = oracle.step_avg(f0, conserved(q), 9, alpha=0.03, chi=chi, variant=variant)
        ref, cf = oracle.step_avg(ref, cf, 6, alpha=0.5, chi=chi, variant=variant)
        assert rel_max(got, ref) <= 1e-12


def test_autotune_keeps_running_mean_reference():
    nx, ny = 130, 40
    rho, ux, uy, chi, q = case(nx, ny, 91)
    lat = lbm.Lattice(nx, ny, rho=rho, ux=ux, uy=uy, storage="f32", variant="II", ux_base=0.04)
    lat.set_sponge(chi, (1.0, 0.04, 0.0))
    lat.set_qref_field(*q)
    lat.set_qref_average(0.1)
    lat.step(5)
    before = (lat.save_state(), np.stack(lat.qref_field()))
    lat.autotune(reps=2)
    assert (lat.save_state() == before[0]).all()
    assert np.array_equal(np.stack(lat.qref_field()), before[1])
    lat.close()


# ------------------------------------------------------------ batches

BATCH_SHAPES = [None, dict(kernel=0, block=256, rows=0), dict(kernel=2, block=128, rows=7),
                dict(kernel=3, block=256, rows=0), dict(kernel=4, block=64, rows=5)]


def batch_member(k, seed, rates):
    """Ragged members of every variant; two in three carry a fixed per-cell
    reference field; with rates, member 1 has non-zero conserved rates (the
    batch then runs the general form of the collision)."""
    g = np.random.default_rng(seed * 100 + k)
    nx, ny = int(g.integers(3, 90)), int(g.integers(3, 70))
    rho, ux, uy, chi, q = case(nx, ny, seed * 100 + k)
    var = ("II", "I", "III", "none", "visc")[k % 5]
    if var == "I":
        chi = np.minimum(chi, 0.1)
    if var == "visc":
        chi = np.minimum(chi, 1.0)
    s = (0.4, 0.3, 0.3) + (1.9,) * 6 if rates and k == 1 else None
    return dict(nx=nx, ny=ny, rho=rho, ux=ux, uy=uy, chi=chi, q=q if k % 3 != 2 else None,
                variant=var, s=s)


def make_batch_member(m, storage):
    kw = dict(s=m["s"]) if m["s"] is not None else {}
    lat = lbm.Lattice(m["nx"], m["ny"], rho=m["rho"], ux=m["ux"], uy=m["uy"], storage=storage,
                      variant=m["variant"], ux_base=0.04, f16_scale=1e-3, **kw)
    lat.set_sponge(m["chi"], (1.0, 0.04, 0.0))
    if m["q"] is not None:
        lat.set_qref_field(*m["q"])
    return lat


@pytest.mark.parametrize("tuning", BATCH_SHAPES)
@pytest.mark.parametrize("storage,rates", [("f64", False), ("f32", False), ("f16", False),
                                           ("f64", True), ("f32", True)])
def test_batch_with_reference_fields_equals_alone_bitwise(storage, rates, tuning):
    """Members with a fixed per-cell reference field, batched beside members
    without one: every batch launch shape (K-step strips of each K, one-step
    tiles; 23 steps = whole launches plus a remainder) gives the bits of the
    member stepped alone, in the default and the general form."""
    say("case: batch with reference fields", storage, rates, tuning)
    members = [batch_member(k, 7, rates) for k in range(10)]
    alone = []
    for m in members:
        lat = make_batch_member(m, storage)
        lat.step(23)
        alone.append(lat.save_state())
        lat.close()
    lats = [make_batch_member(m, storage) for m in members]
    b = lbm.Batch(lats)
    if tuning is not None:
        b.set_tuning(**tuning)
    b.set_min_items(0)  # K-step launches even for this small batch
    b.step(23)
    b.sync()
    for k, (lat, ref) in enumerate(zip(lats, alone)):
        np.testing.assert_array_equal(lat.save_state(), ref, err_msg="member %d" % k)
    b.close()
    for lat in lats:
        lat.close()


def test_batch_takes_a_field_set_after_joining_and_refuses_a_running_mean():
    """A field set on a member between ticks is used from the next tick on
    (bitwise as alone); a running mean or a line source set on a member makes
    the next tick fail before it enqueues anything, and clearing it lets the
    batch go on."""
    members = [batch_member(k, 8, False) for k in range(4)]
    for m in members:
        m["q"] = None
    q = members[1]["q"] = case(members[1]["nx"], members[1]["ny"], 99)[4]
    ref = make_batch_member(dict(members[1], q=None), "f32")
    ref.step(5)
    ref.set_qref_field(*q)
    ref.step(9)
    lats = [make_batch_member(dict(m, q=None), "f32") for m in members]
    b = lbm.Batch(lats)
    b.set_tuning(kernel=4, block=128, rows=0)
    b.set_min_items(0)
    b.step(5)
    b.sync()  # members are the caller's again between a sync and the next tick
    lats[1].set_qref_field(*q)
    b.step(9)
    b.sync()
    np.testing.assert_array_equal(lats[1].save_state(), ref.save_state())
    ref.close()
    before = [lat.save_state() for lat in lats]
    lats[2].set_qref_field(*case(members[2]["nx"], members[2]["ny"], 98)[4])
    lats[2].set_qref_average(0.1)
    with pytest.raises(lbm.LbmError) as e:
        b.step(4)
    assert "running-mean" in str(e.value)
    for lat, st in zip(lats, before):  # nothing ran
        np.testing.assert_array_equal(lat.save_state(), st)
    lats[2].set_qref_average(0.0)
    b.step(4)
    b.sync()
    lats[3].set_line_source((1.0, 1e-4, 0.05, 0.0, 0.0, 0.0))
    with pytest.raises(lbm.LbmError) as e:
        b.step(1)
    assert "line source" in str(e.value)
    lats[3].set_line_source(None)
    b.step(2)
    b.sync()
    b.close()
    for lat in lats:
        lat.close()
