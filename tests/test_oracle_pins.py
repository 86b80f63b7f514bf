"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks. None of them re-types the oracle's own
formula: they check closed forms derived independently, invariants, the
paper's printed matrix and stability thresholds, brute force on tiny grids,
and agreement between the two independent oracle implementations (C time
stepper O1, numpy Von Neumann O2).
"""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.vn as vn

GOLD = os.path.join(os.path.dirname(__file__), "golden")
MRT = oracle.S_MRT_DEFAULT
VARS = ("none", "I", "II", "III")


def paper():
    with open(os.path.join(GOLD, "paper_values.json")) as fh:
        return json.load(fh)


def uniform_state(nx, ny, rho, ux, uy):
    return oracle.feq_field(np.full((ny, nx), rho), np.full((ny, nx), ux), np.full((ny, nx), uy))


def random_state(nx, ny, seed, amp=1e-3, u0=(0.0, 0.0)):
    g = np.random.default_rng(seed)
    rho = 1.0 + amp * g.standard_normal((ny, nx))
    ux = u0[0] + amp * g.standard_normal((ny, nx))
    uy = u0[1] + amp * g.standard_normal((ny, nx))
    f = oracle.feq_field(rho, ux, uy)
    # add a non-equilibrium part so all nine moments are excited
    return f + amp * 0.1 * g.standard_normal(f.shape)


# ------------------------------------------------------------------ transform (App. A.1)

def test_matrix_is_the_papers():
    """Appendix A.1: the oracle's M equals the printed matrix."""
    gold = np.loadtxt(os.path.join(GOLD, "d2q9_M.txt"))
    M, Mi, cx, cy, w = oracle.tables()
    np.testing.assert_array_equal(M, gold)
    np.testing.assert_array_equal(vn.M, gold)


def test_transform_identities():
    """P4: rows of M are orthogonal, M M^T = diag(9,6,6,36,36,12,12,4,4);
    M^-1 from elimination inverts M; velocities satisfy M_{alpha j} = v_j^alpha
    (Section 2.1) and the weights give c_s^2 = 1/3."""
    M, Mi, cx, cy, w = oracle.tables()
    np.testing.assert_array_equal(M @ M.T, np.diag([9, 6, 6, 36, 36, 12, 12, 4, 4]).astype(float))
    np.testing.assert_allclose(Mi @ M, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(Mi, M.T @ np.diag(1 / np.array([9, 6, 6, 36, 36, 12, 12, 4, 4])), atol=1e-16)
    np.testing.assert_array_equal(cx, M[1])
    np.testing.assert_array_equal(cy, M[2])
    assert abs(w.sum() - 1) < 1e-15
    cs2 = (w * cx * cx).sum()
    assert abs((w * cx * cy).sum()) < 1e-16 and abs((w * cy * cy).sum() - cs2) < 1e-16
    # Section 4.2: lambda = c_s / 2 = 0.288675 pins c_s^2 = 1/3
    lam = paper()["lambda_line_source"]["value"]
    assert abs(np.sqrt(cs2) / 2 - lam) < 1e-6


def test_equilibrium_moments_closed_form():
    """P4: M f^eq and M f^L equal the moment equilibria derived by hand from the
    second-order D2Q9 equilibrium (reading of Section 2.1):
    m^eq = (rho, jx, jy, -2rho + 3|j|^2/rho, rho - 3|j|^2/rho, -jx, -jy,
            (jx^2 - jy^2)/rho, jx jy/rho),  m^L = (rho, jx, jy, -2rho, rho, -jx, -jy, 0, 0)."""
    g = np.random.default_rng(1)
    rho = 1 + 0.1 * g.standard_normal(50)
    ux = 0.2 * g.standard_normal(50)
    uy = 0.2 * g.standard_normal(50)
    M, *_ = oracle.tables()
    me = M @ oracle.feq_field(rho, ux, uy)
    ml = M @ oracle.flin_field(rho, ux, uy)
    jx, jy = rho * ux, rho * uy
    q = (jx * jx + jy * jy) / rho
    exp_eq = np.stack([rho, jx, jy, -2 * rho + 3 * q, rho - 3 * q, -jx, -jy,
                       (jx * jx - jy * jy) / rho, jx * jy / rho])
    exp_l = np.stack([rho, jx, jy, -2 * rho, rho, -jx, -jy, 0 * rho, 0 * rho])
    np.testing.assert_allclose(me, exp_eq, atol=2e-15)
    np.testing.assert_allclose(ml, exp_l, atol=2e-15)


# ------------------------------------------------------------------ time stepper invariants

@pytest.mark.parametrize("variant", VARS)
@pytest.mark.parametrize("S", [MRT, vn.bgk(1.7)], ids=["mrt", "bgk"])
def test_conservation_without_sponge(variant, S):
    """P1: with chi = 0 on a periodic box, total mass and momentum are
    constant (conserved moments, eq. eq_conservative)."""
    f = random_state(24, 16, 3)
    M, *_ = oracle.tables()
    tot0 = (M[:3] @ f.reshape(9, -1)).sum(axis=1)
    out = oracle.step(f, 40, s=S, chi=0.0, qref=(1.0, 0.03, 0.0), variant=variant)
    tot1 = (M[:3] @ out.reshape(9, -1)).sum(axis=1)
    # rounding bound: a few ulps of O(1) populations per cell and step
    bound = 9 * np.finfo(float).eps * f[0].size * 40
    np.testing.assert_allclose(tot1, tot0, rtol=0, atol=bound)
    assert np.abs(out - f).max() > 1e-5  # the state did evolve


def _lambda_closed(variant, s_c, chi, n):
    """P2 closed forms for one conserved row (s_c its rate, n its shift)."""
    if variant == "none":
        return 1.0
    if variant == "I":
        return 1 - chi - s_c * n * chi / (1 + n * chi)
    return (1 - chi * (1 - n + n * s_c)) / (1 + n * chi)


@pytest.mark.parametrize("variant", VARS)
@pytest.mark.parametrize("S,n,m", [(MRT, 0.5, 0.5), (vn.bgk(1.9), 0.5, 0.5), (vn.bgk(1.6), 0.3, 0.7)])
def test_uniform_decay_closed_form(variant, S, n, m):
    """P2: a uniform state under uniform chi relaxes to q_ref geometrically,
    c_t - c^f = lambda^t (c_0 - c^f), with lambda derived from the implicit
    rho*, j* definitions of Sections 2.2.1-2.2.3 (sum_i F_i = chi(rho^f - rho*),
    Appendix B.1). For MRT (s_0 = 0) Type I gives 1 - chi and II/III give
    (1 - chi/2)/(1 + chi/2)."""
    chi = 0.1
    qf = (1.0, 0.05, -0.02)
    f = uniform_state(4, 3, 1.01, 0.08, 0.01)
    M, *_ = oracle.tables()
    c0 = M[:3] @ f[:, 0, 0]
    cf = np.array([qf[0], qf[0] * qf[1], qf[0] * qf[2]])
    lam = np.array([_lambda_closed(variant, S[0], chi, n), _lambda_closed(variant, S[1], chi, m),
                    _lambda_closed(variant, S[2], chi, m)])
    cur = f
    for t in range(1, 8):
        cur = oracle.step(cur, 1, s=S, chi=chi, qref=qf, n=n, m=m, variant=variant)
        ct = M[:3] @ cur[:, 0, 0]
        np.testing.assert_allclose(ct - cf, lam ** t * (c0 - cf), rtol=0, atol=1e-14)
    if S is MRT and variant == "I":
        assert abs(lam[0] - 0.9) < 1e-15
    if S is MRT and variant in ("II", "III"):
        assert abs(lam[0] - 0.95 / 1.05) < 1e-15


@pytest.mark.parametrize("variant", VARS)
def test_reference_equilibrium_is_fixed_point(variant):
    """P3: f = f^eq(q_ref) with q_ref = (rho0, u0) is invariant for every
    variant and any chi(x) >= 0 (the rest state is the u0 = 0 case)."""
    g = np.random.default_rng(5)
    # Type I is only stable for s + chi <= 2 (eq. effectrelax); above that the
    # fixed point still holds but rounding noise grows.
    chi = g.uniform(0, 0.1 if variant == "I" else 1.5, (12, 20))
    for q in ((1.0, 0.0, 0.0), (1.0, 0.11547, 0.0), (0.97, 0.05, -0.08)):
        f = uniform_state(20, 12, *q)
        out = oracle.step(f, 25, s=MRT, chi=chi, qref=q, variant=variant)
        assert np.abs(out - f).max() < 4e-15


@pytest.mark.parametrize("S", [MRT, vn.bgk(1.9)], ids=["mrt", "bgk"])
def test_type_I_general_equals_rewritten(S):
    """Section 2.2.1: the general form (f^ref = f^eq(rho^f, u^f), f* = f) equals
    the rewritten form of eq. app:newbgka (rate s' = s + chi, force
    F = chi (f^eq(rho^f,u^f) - f^eq(rho*,u*)))."""
    f = random_state(10, 8, 7, amp=3e-3)
    chi = np.random.default_rng(8).uniform(0, 0.2, (8, 10))
    a = oracle.step(f, 5, s=S, chi=chi, qref=(1.0, 0.05, 0.0), variant="I")
    b = oracle.step(f, 5, s=S, chi=chi, qref=(1.0, 0.05, 0.0), variant="I_rewritten")
    np.testing.assert_allclose(a, b, rtol=0, atol=2e-15)


@pytest.mark.parametrize("variant", VARS)
def test_y_invariance_reduction(variant):
    """P8: a y-uniform state with an x-only sponge evolves exactly like the same
    run on an nx-by-1 periodic lattice (y-streaming wraps onto itself)."""
    nx, ny = 40, 7
    g = np.random.default_rng(11)
    rho = 1 + 1e-3 * np.sin(2 * np.pi * np.arange(nx) / 10)
    f1 = oracle.feq_field(rho[None, :], np.full((1, nx), 0.05), np.full((1, nx), 0.01))
    f1 = f1 + 1e-5 * g.standard_normal(f1.shape)
    fN = np.repeat(f1, ny, axis=1)
    chi_x = np.maximum(0, (8 - np.minimum(np.arange(nx), nx - 1 - np.arange(nx))) / 8) ** 2 * 0.3
    a = oracle.step(f1, 30, s=MRT, chi=chi_x[None, :], qref=(1, 0.05, 0), variant=variant)
    b = oracle.step(fN, 30, s=MRT, chi=np.repeat(chi_x[None, :], ny, axis=0), qref=(1, 0.05, 0), variant=variant)
    for y in range(ny):
        np.testing.assert_array_equal(b[:, y, :], a[:, 0, :])


def test_light_cone_variant_identity():
    """P9: after t steps, cells farther than t (Chebyshev, periodic) from every
    cell with chi > 0 are bitwise identical for all variants; with chi = 0
    everywhere every variant equals the plain scheme bitwise."""
    nx, ny, t = 40, 36, 6
    f = random_state(nx, ny, 13)
    chi = np.zeros((ny, nx))
    chi[2:6, 3:7] = 0.4
    outs = {v: oracle.step(f, t, s=MRT, chi=chi, qref=(1, 0.02, 0), variant=v) for v in VARS}
    ys, xs = np.nonzero(chi)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    dist = np.full((ny, nx), 10 ** 9)
    for y0, x0 in zip(ys, xs):
        dx = np.abs(X - x0)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(Y - y0)
        dy = np.minimum(dy, ny - dy)
        dist = np.minimum(dist, np.maximum(dx, dy))
    far = dist > t
    near = dist <= 1
    for v in ("I", "II", "III"):
        np.testing.assert_array_equal(outs[v][:, far], outs["none"][:, far])
        assert np.abs(outs[v][:, near] - outs["none"][:, near]).max() > 0
    zero = {v: oracle.step(f, t, s=MRT, chi=0.0, qref=(1, 0.02, 0), variant=v) for v in VARS}
    for v in ("I", "II", "III"):
        np.testing.assert_array_equal(zero[v], zero["none"])


def test_bgk_unit_rate_gives_equilibrium():
    """P10: BGK with s = 1 and no sponge collides exactly onto f^eq(rho, j)."""
    g = np.random.default_rng(17)
    fin = oracle.feq_field(1 + 0.01 * g.standard_normal(30), 0.1 * g.standard_normal(30),
                           0.1 * g.standard_normal(30)).T + 1e-3 * g.standard_normal((30, 9))
    out = oracle.collide(fin, s=vn.bgk(1.0), chi=0.0, variant="none")
    M, *_ = oracle.tables()
    mom = fin @ M.T
    expect = oracle.feq_field(mom[:, 0], mom[:, 1] / mom[:, 0], mom[:, 2] / mom[:, 0]).T
    np.testing.assert_allclose(out, expect, rtol=0, atol=1e-15)


def test_shear_wave_decay_rate():
    """P10: at chi = 0 a shear wave u_y = U sin(kx) decays as exp(-nu k^2 t) with
    nu = c_s^2 (1/s - 1/2) (Section 2.2.2 definition of nu; eq. th:d shear mode)."""
    nx, ny = 64, 2
    k = 2 * np.pi / nx
    x = np.arange(nx)
    U = 1e-4
    uy = np.repeat((U * np.sin(k * x))[None, :], ny, axis=0)
    f = oracle.feq_field(np.ones((ny, nx)), np.zeros((ny, nx)), uy)
    s_nu = 1.9
    S = (0, 0, 0, 1.9, 1.9, 1.9, 1.9, s_nu, s_nu)

    def amp(fs):
        _, _, uyy = oracle.moments(fs)
        return 2 * (uyy[0] * np.sin(k * x)).mean()

    f1 = oracle.step(f, 100, s=S, variant="none")
    f2 = oracle.step(f1, 400, s=S, variant="none")
    rate = -np.log(amp(f2) / amp(f1)) / 400
    nu = (1 / 3) * (1 / s_nu - 0.5)
    assert abs(rate / (nu * k * k) - 1) < 2e-3


# ------------------------------------------------------------------ Von Neumann (Section 3.2-3.3)

@pytest.mark.parametrize("variant", VARS)
@pytest.mark.parametrize("q", [(1.0, 0.0, 0.0), (1.03, 0.1, -0.04)])
def test_linearization_closed_form_and_time_stepper(variant, q):
    """The complex-step Jacobian of O2's collision equals the moment-space
    closed form M^-1 A_m M, and O1's collision agrees with it by central
    differences (two independent implementations)."""
    S = MRT
    chi = 0.37
    A = vn.linearized_collision(S, chi, q, variant=variant)
    Am = vn.closed_form_Am(S, chi, q, variant=variant)
    np.testing.assert_allclose(A, vn.MINV @ Am @ vn.M, rtol=0, atol=1e-14)
    f0 = vn.feq(q[0], q[0] * q[1], q[0] * q[2])
    eps = 1e-6
    Af = np.zeros((9, 9))
    for j in range(9):
        fp = f0.copy()
        fp[j] += eps
        fm = f0.copy()
        fm[j] -= eps
        Af[:, j] = (oracle.collide(fp, s=S, chi=chi, qref=q, variant=variant)[0]
                    - oracle.collide(fm, s=S, chi=chi, qref=q, variant=variant)[0]) / (2 * eps)
    np.testing.assert_allclose(Af, A, rtol=0, atol=1e-9)


def _k0_spectrum(variant, S, chi, n, m):
    """P5: exact k = 0 spectrum from the block-triangular A_m."""
    cons = [_lambda_closed(variant, S[0], chi, n), _lambda_closed(variant, S[1], chi, m),
            _lambda_closed(variant, S[2], chi, m)]
    extra = chi if variant == "I" else 0.0
    return np.array(cons + [1 - S[k] - extra for k in range(3, 9)])


@pytest.mark.parametrize("variant", VARS)
@pytest.mark.parametrize("S", [MRT, vn.bgk(1.99)], ids=["mrt", "bgk"])
def test_k0_spectrum_and_det_invariant(variant, S):
    """P5 and P6: the k = 0 spectrum is the closed form; det G(k) = det A for
    every k because sum_j c_j = 0 makes det diag(exp(-i k.c)) = 1."""
    chi, q = 0.45, (1.0, 0.08, 0.03)
    A = vn.linearized_collision(S, chi, q, variant=variant)
    lam0 = np.sort(np.linalg.eigvals(A).real)
    np.testing.assert_allclose(lam0, np.sort(_k0_spectrum(variant, S, chi, 0.5, 0.5)), atol=1e-7)
    detA = np.prod(_k0_spectrum(variant, S, chi, 0.5, 0.5))
    g = np.random.default_rng(19)
    kx, ky = g.uniform(-np.pi, np.pi, (2, 64))
    G = vn.amplification(A, kx, ky)
    dets = np.linalg.det(G)
    np.testing.assert_allclose(dets, detA, rtol=0, atol=1e-13)
    lam = np.linalg.eigvals(G)
    np.testing.assert_allclose(np.prod(lam, axis=1), detA, rtol=0, atol=1e-12)


@pytest.mark.parametrize("s", [1.9, 1.99, 1.99999])
def test_type_II_critical_chi(s):
    """Section 3.1 eq. criticalchi and Section 3.3 Figs. fig:2-fig:4: BGK with
    Type II, n = m = 1/2, theta = 0: stable for chi <= 4/s (|lambda| = 1 exactly
    at chi = 4/s), unstable above."""
    k = np.linspace(-np.pi, np.pi, 241)
    mx = {}
    for d in (-0.1, 0.0, 0.1):
        lam = vn.eigenvalues(vn.bgk(s), 4 / s + d, (1, 0, 0), k, 0 * k, variant="II")
        mx[d] = np.abs(lam).max()
    assert mx[-0.1] < 1 + 1e-12
    assert abs(mx[0.0] - 1) < 1e-12
    assert mx[0.1] > 1.04
    A = vn.linearized_collision(vn.bgk(s), 4 / s, (1, 0, 0), variant="II")
    assert abs(np.linalg.eigvals(A).real.min() + 1) < 1e-12


@pytest.mark.parametrize("n", [0.3, 0.5, 0.7])
def test_general_n_critical_chi(n):
    """Section 3.1 eq. s3rdchi: chi = 2/((1 - 2n + n s) dt) is the exact k = 0
    marginal point of the conserved mode for BGK Types II/III."""
    s = 1.9
    chi_c = 2 / (1 - 2 * n + n * s)
    for variant in ("II", "III"):
        A = vn.linearized_collision(vn.bgk(s), chi_c, (1, 0, 0), n=n, m=n, variant=variant)
        assert abs(np.linalg.eigvals(A).real.min() + 1) < 1e-10


def test_type_I_threshold_cases():
    """Section 2.2.1 eq. effectrelax and Fig. fig:1: Type I is marginally
    stable at s + chi = 2 (s = 1.9, chi = 0.1) and unstable for s = 1.99,
    chi = 0.2."""
    k = np.linspace(-np.pi, np.pi, 241)
    a = np.abs(vn.eigenvalues(vn.bgk(1.9), 0.1, (1, 0, 0), k, 0 * k, variant="I")).max()
    b = np.abs(vn.eigenvalues(vn.bgk(1.99), 0.2, (1, 0, 0), k, 0 * k, variant="I")).max()
    assert abs(a - 1) < 1e-12
    assert abs(b - 1.19) < 1e-9


def test_mean_flow_claims():
    """Section 3.3, Figs. fig:8 and fig:9, u^f = (0.1, 0), s = 1.99: Type II keeps
    its critical chi (stable at 4/s - 0.1); Type III is not stable at 4/s - 0.1
    and its critical chi lies below 3/s."""
    s = 1.99
    k = np.linspace(-np.pi, np.pi, 401)
    q = (1.0, 0.1, 0.0)
    ii = np.abs(vn.eigenvalues(vn.bgk(s), 4 / s - 0.1, q, k, 0 * k, variant="II")).max()
    ii_hi = np.abs(vn.eigenvalues(vn.bgk(s), 4 / s + 0.1, q, k, 0 * k, variant="II")).max()
    iii = np.abs(vn.eigenvalues(vn.bgk(s), 4 / s - 0.1, q, k, 0 * k, variant="III")).max()
    iii3 = np.abs(vn.eigenvalues(vn.bgk(s), 3 / s, q, k, 0 * k, variant="III")).max()
    assert ii < 1 + 1e-12 and ii_hi > 1.01
    assert iii > 1.01 and iii3 > 1 + 1e-4


def test_acoustic_and_shear_modes_small_k():
    """Eq. th:d at chi = 0 and small k: acoustic Re omega = |k|(+-c_s + |u| cos),
    shear Re omega = |k||u| cos and Im omega = -nu |k|^2 (theta = 0)."""
    s = 1.9
    nu = (1 / 3) * (1 / s - 0.5)
    cs = np.sqrt(1 / 3)
    k = 0.01
    for ux in (0.0, 0.1):
        lam = vn.eigenvalues(vn.bgk(s), 0.0, (1, ux, 0), [k], [0.0], variant="none")[0]
        hyd = lam[np.abs(lam - 1) < 0.5]
        assert hyd.size == 3
        omega = 1j * np.log(hyd)  # lambda = exp(-i omega)
        re = np.sort(omega.real)
        np.testing.assert_allclose(re, np.sort([k * (-cs + ux), k * ux, k * (cs + ux)]), rtol=2e-3, atol=1e-7)
        if ux == 0.0:
            # with mean flow D2Q9 carries an O(u^2) viscosity defect
            # (Galilean invariance), so the damping is checked at rest only
            shear = omega[np.argmin(np.abs(omega.real - k * ux))]
            assert abs(shear.imag / (-nu * k * k) - 1) < 2e-3


@pytest.mark.parametrize("variant", ["I", "II", "III"])
def test_brute_force_dft_matches_vn_matrix(variant):
    """P7: one O1 step from f^eq(q^f) +- eps e_j at one cell, central
    differences, and a DFT over the periodic lattice give column j of G(k) at
    every lattice wavenumber; it must equal O2's G(k)."""
    nx, ny = 8, 6
    chi, q, S = 0.3, (1.0, 0.06, -0.03), MRT
    base = uniform_state(nx, ny, *q)
    eps = 1e-5  # central-difference truncation O(eps^2) ~ 1e-10
    A = vn.linearized_collision(S, chi, q, variant=variant)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    KX, KY = np.meshgrid(kx, ky)
    G = vn.amplification(A, KX.ravel(), KY.ravel()).reshape(ny, nx, 9, 9)
    for j in range(9):
        fp = base.copy()
        fp[j, 0, 0] += eps
        fm = base.copy()
        fm[j, 0, 0] -= eps
        dp = oracle.step(fp, 1, s=S, chi=chi, qref=q, variant=variant)
        dm = oracle.step(fm, 1, s=S, chi=chi, qref=q, variant=variant)
        resp = (dp - dm) / (2 * eps)  # [9][ny][nx]
        col = np.fft.fft2(resp, axes=(1, 2))  # sum_x resp(x) exp(-i k.x)
        np.testing.assert_allclose(np.moveaxis(col, 0, -1), G[:, :, :, j], rtol=0, atol=1e-9)


def test_multi_step_mode_evolution():
    """P7 (multi-step): seeding an eigenvector of G(k) and running T steps of
    O1 multiplies its Fourier coefficient by lambda^T."""
    nx, ny, T = 16, 8, 25
    chi, q, S = 0.2, (1.0, 0.05, 0.0), MRT
    A = vn.linearized_collision(S, chi, q, variant="II")
    kx, ky = 2 * np.pi * 3 / nx, 2 * np.pi * 1 / ny
    G = vn.amplification(A, [kx], [ky])[0]
    lam, vec = np.linalg.eig(G)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    phase = np.exp(1j * (kx * X + ky * Y))
    base = uniform_state(nx, ny, *q)
    eps = 1e-6
    for i in np.argsort(-np.abs(lam))[:4]:
        pert = np.real(vec[:, i][:, None, None] * phase[None])
        up = oracle.step(base + eps * pert, T, s=S, chi=chi, qref=q, variant="II")
        dn = oracle.step(base - eps * pert, T, s=S, chi=chi, qref=q, variant="II")
        lin = (up - dn) / (2 * eps)
        coef = (lin * np.conj(phase)[None]).sum(axis=(1, 2)) / (nx * ny / 2)
        np.testing.assert_allclose(coef, lam[i] ** T * vec[:, i], rtol=0, atol=1e-7)


# ------------------------------------------------------------------ viscosity-ramp strategy (Sec. 4.1)

def test_viscosity_ramp_limits():
    """The comparison strategy of Section 4.1 (rates ramped linearly to 1 in
    the layer): at xi = 0 it is the plain scheme bit for bit; at xi = 1 every
    non-conserved moment relaxes fully, so one collision lands exactly on
    f^eq(rho, j) (the BGK s = 1 limit); in between, a uniform state keeps its
    conserved moments and its non-conserved moments relax by 1 - s'."""
    f = random_state(12, 10, 41)
    S = (0.0, 0.0, 0.0, 1.5, 1.6, 1.7, 1.8, 1.9, 1.95)
    a = oracle.step(f, 7, s=S, chi=0.0, variant="visc")
    b = oracle.step(f, 7, s=S, chi=0.0, variant="none")
    np.testing.assert_array_equal(a, b)
    M, *_ = oracle.tables()
    fin = f[:, 0, :].T
    out = oracle.collide(fin, s=S, chi=1.0, variant="visc")
    mom = fin @ M.T
    expect = oracle.feq_field(mom[:, 0], mom[:, 1] / mom[:, 0], mom[:, 2] / mom[:, 0]).T
    np.testing.assert_allclose(out, expect, rtol=0, atol=1e-15)
    xi = 0.3
    out = oracle.collide(fin, s=S, chi=xi, variant="visc")
    m_in, m_out = fin @ M.T, out @ M.T
    meq = oracle.feq_field(m_in[:, 0], m_in[:, 1] / m_in[:, 0], m_in[:, 2] / m_in[:, 0]).T @ M.T
    np.testing.assert_allclose(m_out[:, :3], m_in[:, :3], rtol=0, atol=1e-15)
    for k in range(3, 9):
        sk = S[k] + (1 - S[k]) * xi
        np.testing.assert_allclose(m_out[:, k] - meq[:, k], (1 - sk) * (m_in[:, k] - meq[:, k]),
                                   rtol=0, atol=1e-15)


# ------------------------------------------------------------------ time-averaged reference state (Sec. 1, Sec. 2.2)

def _conserved(f):
    rho, ux, uy = oracle.moments(f)
    return np.stack([rho, rho * ux, rho * uy])


def _qref_field(cf):
    return np.stack([cf[0], cf[1] / cf[0], cf[2] / cf[0]])


def test_averaged_reference_alpha_zero_is_static_field():
    """alpha = 0 keeps the mean fixed: the averaged stepper equals the static
    per-cell reference stepper (up to the rounding of u^f = j^f / rho^f)."""
    f = random_state(11, 9, 52)
    g = np.random.default_rng(53)
    cf = np.stack([1 + 1e-3 * g.standard_normal((9, 11)), 0.05 + 1e-3 * g.standard_normal((9, 11)),
                   1e-3 * g.standard_normal((9, 11))])
    chi = g.uniform(0, 0.4, (9, 11))
    for var in ("I", "II", "III"):
        c_ = np.minimum(chi, 0.1) if var == "I" else chi
        a, cf_out = oracle.step_avg(f, cf, 6, alpha=0.0, chi=c_, variant=var)
        b = oracle.step(f, 6, chi=c_, qref_field=_qref_field(cf), variant=var)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
        np.testing.assert_array_equal(cf_out, cf)


def test_averaged_reference_without_sponge_is_running_mean_of_moments():
    """With chi = 0 the reference never enters the step: populations are those
    of the plain scheme bit for bit, and the mean is the exponential running
    mean of the cell's pre-collision moments over the step history."""
    f = random_state(10, 12, 54)
    cf0 = _conserved(f) * 0.9
    alpha = 0.3
    a, cf = oracle.step_avg(f, cf0, 8, alpha=alpha, chi=0.0, variant="II")
    np.testing.assert_array_equal(a, oracle.step(f, 8, chi=0.0, variant="II"))
    mean, ft = cf0.copy(), f
    for _ in range(8):
        mean = (1 - alpha) * mean + alpha * _conserved(ft)
        ft = oracle.step(ft, 1, chi=0.0, variant="II")
    np.testing.assert_allclose(cf, mean, rtol=0, atol=1e-14)


def test_averaged_reference_equals_static_steps_plus_mean_update():
    """With a sponge, each averaged step is one static-reference step with the
    current mean, followed by the mean update from the pre-collision
    moments; checked for every variant and several rates."""
    f = random_state(9, 8, 55)
    g = np.random.default_rng(56)
    chi = g.uniform(0, 0.3, (8, 9))
    for var in ("I", "II", "III", "none"):
        c_ = np.minimum(chi, 0.1) if var == "I" else chi
        for alpha in (0.05, 0.5, 1.0):
            cf0 = _conserved(f) + 1e-4 * g.standard_normal((3, 8, 9))
            a, cf = oracle.step_avg(f, cf0, 5, alpha=alpha, chi=c_, variant=var)
            ft, mean = f, cf0.copy()
            for _ in range(5):
                nxt = oracle.step(ft, 1, chi=c_, qref_field=_qref_field(mean), variant=var)
                mean = mean + alpha * (_conserved(ft) - mean)
                ft = nxt
            np.testing.assert_allclose(a, ft, rtol=0, atol=1e-14)
            np.testing.assert_allclose(cf, mean, rtol=0, atol=1e-14)


def test_averaged_reference_equilibrium_is_fixed_point():
    """A uniform equilibrium whose mean equals its own state stays fixed for
    every variant, rate and sponge."""
    n = 7
    rho = np.full((n, n), 1.01)
    ux = np.full((n, n), 0.06)
    uy = np.full((n, n), -0.02)
    f0 = oracle.feq_field(rho, ux, uy)
    cf0 = np.stack([rho, rho * ux, rho * uy])
    chi = np.random.default_rng(57).uniform(0, 0.5, (n, n))
    for var in ("I", "II", "III"):
        a, cf = oracle.step_avg(f0, cf0, 10, alpha=0.2, chi=np.minimum(chi, 0.1) if var == "I"
                                else chi, variant=var)
        np.testing.assert_allclose(a, f0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(cf, cf0, rtol=0, atol=1e-15)


# ------------------------------------------------------------------ line source and outflow (Sec. 4.2)

SRC = (1.0, 1e-4, 0.01, 0.3, 0.04, 0.0)   # rho0, amp, freq (per step), phase, ux, uy


def _rho_src(t, src=SRC):
    return src[0] + src[1] * np.sin(2 * np.pi * src[2] * t + src[3])


def test_line_source_injects_the_source_equilibrium():
    """After a step from time t0, the populations moving in +x at x = 1 are
    those of the source equilibrium f^eq(rho_src(t0 + 1), u_src) (closed form,
    any state, any sponge, any variant)."""
    f = random_state(12, 7, 61, u0=(0.04, 0.0))
    chi = np.random.default_rng(62).uniform(0, 0.3, (7, 12))
    for var, t0 in (("II", 0), ("III", 17), ("none", 5)):
        out = oracle.step_line_source(f, 1, source=SRC, t0=t0, chi=chi, variant=var,
                                      qref=(1.0, 0.04, 0.0))
        rs = _rho_src(t0 + 1)
        feq = oracle.feq_field(np.full((7, 1), rs), np.full((7, 1), SRC[4]),
                               np.full((7, 1), SRC[5]))
        for i in (1, 5, 8):
            np.testing.assert_allclose(out[i, :, 1], feq[i, :, 0], rtol=0, atol=1e-16)


def test_line_source_outflow_copies_the_last_interior_column():
    """With outflow, the populations moving in -x at x = nx - 2 after a step
    are the post-collision populations of column nx - 2 itself (pulled from
    column nx - 1, which holds its copy)."""
    nx, ny = 10, 6
    f = random_state(nx, ny, 63, u0=(0.04, 0.0))
    M, _, cx, cy, _ = oracle.tables()
    out = oracle.step_line_source(f, 1, source=SRC, variant="II", qref=(1.0, 0.04, 0.0))
    post = oracle.collide(f[:, :, nx - 2].T, variant="II", qref=(1.0, 0.04, 0.0)).T  # [9][ny]
    for i in (3, 6, 7):
        np.testing.assert_allclose(out[i, :, nx - 2], np.roll(post[i], int(cy[i])), rtol=0,
                                   atol=1e-16)


def test_line_source_outflow_is_local():
    """The outflow column influences the channel at most one cell per step:
    a channel twice as long gives the same populations on x < nx - 1 - T."""
    nx, ny, T = 40, 5, 15
    f = random_state(2 * nx, ny, 64, u0=(0.04, 0.0))
    short = oracle.step_line_source(f[:, :, :nx], T, source=SRC, variant="II",
                                    qref=(1.0, 0.04, 0.0))
    long_ = oracle.step_line_source(f, T, source=SRC, variant="II", qref=(1.0, 0.04, 0.0))
    np.testing.assert_array_equal(short[:, :, 1:nx - 1 - T], long_[:, :, 1:nx - 1 - T])


def test_line_source_y_invariance():
    """A y-uniform state with the y-uniform source keeps every row equal to
    the one-row channel."""
    nx = 30
    row = random_state(nx, 1, 65, u0=(0.04, 0.0))
    f = np.repeat(row, 6, axis=1)
    a = oracle.step_line_source(f, 40, source=SRC, variant="II", qref=(1.0, 0.04, 0.0),
                                chi=np.tile(np.linspace(0, 0.3, nx), (6, 1)))
    b = oracle.step_line_source(row, 40, source=SRC, variant="II", qref=(1.0, 0.04, 0.0),
                                chi=np.linspace(0, 0.3, nx)[None, :])
    for y in range(6):
        np.testing.assert_array_equal(a[:, y], b[:, 0])


@pytest.mark.parametrize("u0", [0.0, 0.1])
def test_line_source_emits_the_acoustic_wavelength(u0):
    """The source emits a plane wave of wavelength (c_s + u0) / freq: the mean
    spacing of the downward zero crossings of rho' behind the front matches
    it within 2% (freq = 0.01 per step, as in the paper's set-up)."""
    nx, T = 600, 420
    src = (1.0, 1e-4, 0.01, 0.0, u0, 0.0)
    rho = np.ones((1, nx))
    f0 = oracle.feq_field(rho, np.full((1, nx), u0), np.zeros((1, nx)))
    S = (0.0, 0.0, 0.0) + (1.9988,) * 6
    f = oracle.step_line_source(f0, T, source=src, s=S, variant="none", qref=(1.0, u0, 0.0))
    rp = f.sum(axis=0)[0] - 1.0
    cs = 1 / np.sqrt(3)
    front = int((cs + u0) * T)
    seg = rp[5:front - 40]
    down = np.where((seg[:-1] > 0) & (seg[1:] <= 0))[0]
    x0 = down + seg[down] / (seg[down] - seg[down + 1])   # linear interpolation
    lam = np.diff(x0).mean()
    assert abs(lam / ((cs + u0) / 0.01) - 1) < 0.02, lam

