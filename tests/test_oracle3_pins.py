"""Pins of the D3Q15 oracle (Appendix A.2; the scheme of Section 2 in three
dimensions) against what the paper and the mathematics fix: the printed
matrix, orthogonality, lattice isotropy, the equilibrium moments of the
D3Q15 MRT model, conservation, the closed-form decay of a uniform state
towards q_ref, the reference fixed point, z-invariance, the light cone, the
BGK s = 1 limit and the shear viscosity nu = c_s^2 (1/s - 1/2)."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle.d3q15 as o3

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d3q15_M.txt")
CS2 = 1.0 / 3.0


def random_state(nx, ny, nz, seed, amp=1e-3, u0=(0.0, 0.0, 0.0)):
    g = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = 1 + amp * g.standard_normal(shape)
    u = [u0[k] + amp * g.standard_normal(shape) for k in range(3)]
    f = o3.feq_field(rho, *u)
    return f + 0.1 * amp * g.standard_normal(f.shape)


def test_matrix_is_the_papers():
    M = o3.tables()[0]
    np.testing.assert_array_equal(M, np.loadtxt(GOLDEN))


def test_rows_are_orthogonal():
    M = o3.tables()[0]
    G = M @ M.T
    np.testing.assert_array_equal(G, np.diag(np.diag(G)))
    np.testing.assert_array_equal(np.diag(G), [15, 10, 10, 10, 18, 360, 40, 40, 40, 12, 4, 8, 8, 8, 8])
    Mi = o3.tables()[1]
    np.testing.assert_allclose(Mi, M.T / np.diag(G), rtol=0, atol=1e-15)


def test_velocities_and_weights_are_isotropic():
    _, _, cx, cy, cz, w = o3.tables()
    c = np.stack([cx, cy, cz]).astype(float)
    assert set(map(tuple, c.T.astype(int))) == ({(0, 0, 0)} | {tuple(v) for v in np.eye(3, dtype=int)}
                                                | {tuple(-v) for v in np.eye(3, dtype=int)}
                                                | set(itertools.product((-1, 1), repeat=3)))
    assert abs(w.sum() - 1) < 1e-15
    d = np.eye(3)
    np.testing.assert_allclose(np.einsum("i,ai->a", w, c), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ai,bi->ab", w, c, c), d / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ai,bi,ci->abc", w, c, c, c), 0, atol=1e-16)
    four = np.einsum("i,ai,bi,ci,di->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(four, iso, atol=1e-16)


def test_equilibrium_moments_are_the_d3q15_mrt_ones():
    """M f^eq(rho, j) = (rho, j, -rho + j^2/rho, rho - 5 j^2/rho, -7/3 j,
    (2jx^2 - jy^2 - jz^2)/rho, (jy^2 - jz^2)/rho, jx jy/rho, jy jz/rho,
    jz jx/rho, 0) and the linear part drops every term in j^2/rho."""
    M = o3.tables()[0]
    g = np.random.default_rng(3)
    for _ in range(5):
        rho = 1 + 0.1 * g.standard_normal()
        u = 0.1 * g.standard_normal(3)
        jx, jy, jz = rho * u
        j2 = (jx * jx + jy * jy + jz * jz) / rho
        expect = [rho, jx, jy, jz, -rho + j2, rho - 5 * j2, -7 / 3 * jx, -7 / 3 * jy, -7 / 3 * jz,
                  (2 * jx * jx - jy * jy - jz * jz) / rho, (jy * jy - jz * jz) / rho,
                  jx * jy / rho, jy * jz / rho, jz * jx / rho, 0.0]
        feq = o3.feq_field(np.array([rho]), u[0], u[1], u[2])[:, 0]
        np.testing.assert_allclose(M @ feq, expect, rtol=0, atol=1e-14)


def test_conservation_without_sponge():
    f = random_state(7, 6, 5, 1, u0=(0.03, -0.02, 0.01))
    g = o3.step(f, 20, chi=0.0, variant="II")
    rho0, *u0 = o3.moments(f)
    rho1, *u1 = o3.moments(g)
    tol = 1e-15 * f.size * 20
    assert abs(rho1.sum() - rho0.sum()) < tol
    for a, b, r0, r1 in zip(u0, u1, [rho0] * 3, [rho1] * 3):
        assert abs((r1 * b).sum() - (r0 * a).sum()) < tol


@pytest.mark.parametrize("variant", ["I", "II", "III"])
def test_reference_state_is_a_fixed_point(variant):
    n = 5
    q = (1.01, 0.05, -0.02, 0.03)
    f0 = o3.feq_field(np.full((n, n, n), q[0]), q[1], q[2], q[3])
    chi = np.random.default_rng(4).uniform(0, 0.1 if variant == "I" else 0.5, (n, n, n))
    f = o3.step(f0, 10, chi=chi, qref=q, variant=variant)
    np.testing.assert_allclose(f, f0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("variant", ["I", "II", "III"])
@pytest.mark.parametrize("nn,mm", [(0.5, 0.5), (0.3, 0.8)])
def test_uniform_state_decays_towards_the_reference(variant, nn, mm):
    """A uniform state relaxes its conserved moments towards c^f by a
    closed-form factor per step: 1 - chi for Type I; (1 + (p - 1) chi) /
    (1 + p chi) for Types II and III, p = n for rho and p = m for j
    (the shifted state c* = (c + p chi c^f)/(1 + p chi) meets the damping
    chi (c^f - c*))."""
    N, T, chi = 3, 7, 0.08
    q = (1.0, 0.02, 0.0, -0.01)
    f = o3.feq_field(np.full((N, N, N), 1.002), 0.025, 0.004, -0.013)
    g = o3.step(f, T, chi=chi, qref=q, variant=variant, n=nn, m=mm)
    M = o3.tables()[0]
    m0 = np.einsum("ki,izyx->k", M, f[:, :1, :1, :1])
    m1 = np.einsum("ki,izyx->k", M, g[:, :1, :1, :1])
    cf = np.array([q[0], q[0] * q[1], q[0] * q[2], q[0] * q[3]])
    if variant == "I":
        fac = np.full(4, 1 - chi)
    else:
        fac = np.array([(1 + (p - 1) * chi) / (1 + p * chi) for p in (nn, mm, mm, mm)])
    np.testing.assert_allclose(m1[:4] - cf, (m0[:4] - cf) * fac ** T, rtol=1e-11, atol=1e-16)


def test_free_streaming_moves_each_population_by_its_velocity():
    """With every rate and the sponge at zero the collision is the identity
    (M^-1 M f, exact up to rounding), so T steps move population i by T c_i
    (periodic)."""
    f = random_state(7, 6, 5, 9)
    T = 3
    g = o3.step(f, T, s=(0.0,) * 15, chi=0.0, variant="none")
    _, _, cx, cy, cz, _ = o3.tables()
    for i in range(15):
        expect = np.roll(f[i], (T * cz[i], T * cy[i], T * cx[i]), axis=(0, 1, 2))
        np.testing.assert_allclose(g[i], expect, rtol=0, atol=1e-15)


def test_z_invariance_reduces_to_one_plane():
    f2 = random_state(9, 8, 1, 5, u0=(0.04, 0.0, 0.0))
    f = np.repeat(f2, 4, axis=1)
    chi2 = np.random.default_rng(6).uniform(0, 0.3, (1, 8, 9))
    a = o3.step(f, 12, chi=np.repeat(chi2, 4, axis=0), qref=(1.0, 0.04, 0.0, 0.0))
    b = o3.step(f2, 12, chi=chi2, qref=(1.0, 0.04, 0.0, 0.0))
    for z in range(4):
        np.testing.assert_array_equal(a[:, z], b[:, 0])


def test_light_cone():
    """A point perturbation reaches at most T cells along each axis in T steps."""
    n, T = 15, 4
    f0 = o3.feq_field(np.ones((n, n, n)), 0.0, 0.0, 0.0)
    f = f0.copy()
    f[:, 7, 7, 7] += 1e-4 * np.random.default_rng(7).standard_normal(15)
    d = np.abs(o3.step(f, T, chi=0.0) - o3.step(f0, T, chi=0.0)).max(axis=0)
    nz_ = np.argwhere(d > 0)
    assert nz_.size and np.abs(nz_ - 7).max() <= T
    assert d[7, 7, 7 + T] > 0 or d[7, 7 + T, 7] > 0 or d[7 + T, 7, 7] > 0


def test_bgk_unit_rates_land_on_the_equilibrium():
    f = random_state(4, 3, 2, 8).reshape(15, -1).T
    S = (0.0,) * 4 + (1.0,) * 11
    out = o3.collide(f, s=S, chi=0.0, variant="none")
    M = o3.tables()[0]
    m = f @ M.T
    feq = o3.feq_field(m[:, 0], m[:, 1] / m[:, 0], m[:, 2] / m[:, 0], m[:, 3] / m[:, 0]).T
    np.testing.assert_allclose(out, feq, rtol=0, atol=1e-15)


@pytest.mark.parametrize("s", [1.2, 1.7])
def test_shear_wave_decays_at_the_mrt_viscosity(s):
    """u_x = U sin(k y): the mode decays as exp(-nu k^2 t) with
    nu = c_s^2 (1/s - 1/2) (s the rate of the stress rows), to leading order
    in k: within 1% for a 128-cell wavelength (the scheme's higher-order
    dispersion shifts it by O(k^2))."""
    L, T = 128, 800
    y = np.arange(L)
    k = 2 * np.pi / L
    ux = 1e-4 * np.sin(k * y)[None, :, None] * np.ones((2, L, 2))
    f0 = o3.feq_field(np.ones((2, L, 2)), ux, 0.0, 0.0)
    S = (0.0,) * 4 + (s,) * 11
    f = o3.step(f0, T, s=S, chi=0.0, variant="none")
    _, u1, _, _ = o3.moments(f)
    amp0 = (ux[0, :, 0] * np.sin(k * y)).sum()
    amp1 = (u1[0, :, 0] * np.sin(k * y)).sum()
    nu = CS2 * (1 / s - 0.5)
    assert abs(math.log(amp1 / amp0) / (-nu * k * k * T) - 1) < 1e-2


# ------------------------------------------------------------------ viscosity-ramp strategy (Sec. 4.1 on App. A.2)

S_RAMP = (0.0,) * 4 + (1.1, 1.25, 1.4, 1.5, 1.6, 1.7, 1.75, 1.8, 1.85, 1.9, 1.95)


def _meq_of_input(fin):
    """M f^eq(rho, j) of each input cell's own conserved moments."""
    M = o3.tables()[0]
    m = fin @ M.T
    feq = o3.feq_field(m[:, 0], m[:, 1] / m[:, 0], m[:, 2] / m[:, 0], m[:, 3] / m[:, 0]).T
    return m, feq, feq @ M.T


def test_viscosity_ramp_at_zero_is_the_plain_scheme():
    """The comparison strategy of Sec. 4.1 (non-conserved rates ramped
    linearly to 1 across the layer) with the ramp coordinate 0 everywhere is
    the undamped scheme bit for bit."""
    f = random_state(6, 5, 4, 21, u0=(0.03, 0.0, -0.02))
    a = o3.step(f, 6, s=S_RAMP, chi=0.0, variant="visc")
    b = o3.step(f, 6, s=S_RAMP, chi=0.0, variant="none")
    np.testing.assert_array_equal(a, b)


def test_viscosity_ramp_at_one_lands_on_the_equilibrium():
    """At ramp coordinate 1 every non-conserved rate is 1, so one collision
    lands exactly on f^eq(rho, j) of the cell (the BGK s = 1 limit)."""
    fin = random_state(4, 3, 2, 22, u0=(0.05, -0.03, 0.02)).reshape(15, -1).T
    out = o3.collide(fin, s=S_RAMP, chi=1.0, variant="visc", qref=(1.3, 0.2, 0.1, 0.0))
    _, feq, _ = _meq_of_input(fin)
    np.testing.assert_allclose(out, feq, rtol=0, atol=1e-15)


@pytest.mark.parametrize("xi", [0.3, 0.75])
def test_viscosity_ramp_relaxes_each_moment_at_the_ramped_rate(xi):
    """In between, the conserved moments are kept (no force: q_ref and chi
    play no part), and each non-conserved moment k moves from its value
    towards m^eq_k by the ramped rate s'_k = s_k + (1 - s_k) xi:
    m'_k - m^eq_k = (1 - s'_k)(m_k - m^eq_k)."""
    fin = random_state(4, 3, 2, 23, u0=(-0.04, 0.02, 0.06)).reshape(15, -1).T
    M = o3.tables()[0]
    out = o3.collide(fin, s=S_RAMP, chi=xi, variant="visc", qref=(0.8, -0.1, 0.0, 0.2))
    m_in, _, meq = _meq_of_input(fin)
    m_out = out @ M.T
    np.testing.assert_allclose(m_out[:, :4], m_in[:, :4], rtol=0, atol=1e-15)
    for k in range(4, 15):
        sk = S_RAMP[k] + (1 - S_RAMP[k]) * xi
        np.testing.assert_allclose(m_out[:, k] - meq[:, k], (1 - sk) * (m_in[:, k] - meq[:, k]),
                                   rtol=0, atol=1e-14)


def test_viscosity_ramp_uniform_state_decay():
    """A uniform state (wavenumber 0, streaming moves nothing) under a uniform
    ramp coordinate: its conserved moments stay, so m^eq stays, and after T
    steps each non-conserved moment's distance to m^eq has shrunk by
    (1 - s'_k)^T."""
    xi, T = 0.4, 5
    base = o3.feq_field(np.full((2, 2, 2), 1.01), 0.04, -0.02, 0.03)
    kick = np.random.default_rng(24).standard_normal(15) * 3e-3
    f = base + kick[:, None, None, None]
    g = o3.step(f, T, s=S_RAMP, chi=xi, variant="visc")
    M = o3.tables()[0]
    m0, _, meq = _meq_of_input(f[:, :1, :1, :1].reshape(15, 1).T)
    m1 = g[:, :1, :1, :1].reshape(15, 1).T @ M.T
    np.testing.assert_allclose(m1[0, :4], m0[0, :4], rtol=0, atol=1e-14)
    for k in range(4, 15):
        sk = S_RAMP[k] + (1 - S_RAMP[k]) * xi
        np.testing.assert_allclose(m1[0, k] - meq[0, k], (1 - sk) ** T * (m0[0, k] - meq[0, k]),
                                   rtol=0, atol=1e-14)
