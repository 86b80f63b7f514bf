"""Von Neumann oracle (O2) for the linearised lattice Boltzmann scheme with an
absorbing term, Section 3.2 (eqs. eq:linearized, perturb-w-f, sec:matrix).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
benchmark's CPU-baseline leg.

The collision is written here a second time, in numpy, so that it accepts
complex arguments. Its Jacobian at the reference state f^eq(rho^f, u^f) is
taken by complex-step differentiation (exact to rounding), which is the
linearisation of eq. eq:linearized including the dependence of rho*, u* on f
through the implicit Guo-type definition. The streaming phase that the
printed eigenproblem omits is restored (pull form): with
delta f_j = A_j exp[i(k.x - omega t)] and delta f_i(x + c_i, t+1) =
sum_j A_ij delta f_j(x, t) one gets

    exp(-i omega) a = G(k) a,   G(k) = diag(exp(-i k.c_i)) A.

Eigenvalues lambda = exp(-i omega): Re omega = -arg lambda,
Im omega = ln |lambda| (growth if > 0).

``closed_form_Am`` gives the same linearisation in moment space,
A = M^-1 A_m M with A_m = I + S (J D P - I) - chi X, which the tests pin
against the complex-step Jacobian.
"""
from __future__ import annotations

import numpy as np

# Appendix A.1
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=np.float64)
CX = M[1].copy()
CY = M[2].copy()
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
MINV = np.linalg.inv(M)

VARIANTS = {"none": 0, "I": 1, "II": 2, "III": 3}


def feq(rho, jx, jy):
    """f^eq(rho, j): second-order D2Q9 equilibrium, any dtype, shape (9, ...)."""
    cj = CX.reshape((9,) + (1,) * np.ndim(rho)) * jx + CY.reshape((9,) + (1,) * np.ndim(rho)) * jy
    w = W.reshape((9,) + (1,) * np.ndim(rho))
    return w * (rho + 3 * cj + 4.5 * cj * cj / rho - 1.5 * (jx * jx + jy * jy) / rho)


def flin(rho, jx, jy):
    cj = CX.reshape((9,) + (1,) * np.ndim(rho)) * jx + CY.reshape((9,) + (1,) * np.ndim(rho)) * jy
    w = W.reshape((9,) + (1,) * np.ndim(rho))
    return w * (rho + 3 * cj)


def collide(f, s, chi, qref, n=0.5, m=0.5, variant="II"):
    """Collision of one cell (no streaming); ``f`` shape (9,), real or complex.

    Sections 2.2.1-2.2.3 with Gamma = chi I; rho*, j* solved exactly from
    their implicit definitions.
    """
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    s = np.asarray(s, dtype=np.float64)
    rf, uxf, uyf = qref
    if v == 0:  # no absorbing term: no force, rho* = rho, j* = j
        chi = 0.0
    mom = M @ f
    rho, jx, jy = mom[0], mom[1], mom[2]
    jxf, jyf = rf * uxf, rf * uyf
    rhos = (rho + n * chi * rf) / (1 + n * chi)
    jxs = (jx + m * chi * jxf) / (1 + m * chi)
    jys = (jy + m * chi * jyf) / (1 + m * chi)
    meqs = M @ feq(rhos, jxs, jys)
    if v == 0:
        d = 0 * mom
    elif v == 1:
        d = chi * (M @ feq(rf, jxf, jyf) - mom)
    elif v == 2:
        d = chi * (M @ feq(rf, jxf, jyf) - meqs)
    elif v == 3:
        d = chi * (M @ flin(rf, jxf, jyf) - M @ flin(rhos, jxs, jys))
    else:
        raise ValueError(variant)
    mp = mom + s * (meqs - mom) + d
    return MINV @ mp


def linearized_collision(s, chi, qref, n=0.5, m=0.5, variant="II", h=1e-30):
    """A_ij = d C_i / d f_j at f = f^eq(q_ref), by complex-step differentiation."""
    rf, uxf, uyf = qref
    f0 = feq(rf, rf * uxf, rf * uyf)
    A = np.empty((9, 9))
    for j in range(9):
        fp = f0.astype(np.complex128)
        fp[j] += 1j * h
        A[:, j] = np.imag(collide(fp, s, chi, qref, n, m, variant)) / h
    return A


def closed_form_Am(s, chi, qref, n=0.5, m=0.5, variant="II"):
    """Moment-space linearisation A_m = I + S (J D P - I) - chi X.

    P projects onto (rho, jx, jy); D = diag(1/(1+n chi), 1/(1+m chi), 1/(1+m chi))
    is the derivative of (rho*, j*) with respect to (rho, j); J = d m^eq / d(rho, j)
    at q_ref; X = I (Type I), J D P (Type II), L D P (Type III, L = d m^L/d(rho, j)).
    """
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    if v == 0:
        chi = 0.0
    rf, ux, uy = qref
    u2 = ux * ux + uy * uy
    J = np.array([
        [1, 0, 0], [0, 1, 0], [0, 0, 1],
        [-2 - 3 * u2, 6 * ux, 6 * uy],
        [1 + 3 * u2, -6 * ux, -6 * uy],
        [0, -1, 0], [0, 0, -1],
        [-(ux * ux - uy * uy), 2 * ux, -2 * uy],
        [-ux * uy, uy, ux]], dtype=np.float64)
    L = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-2, 0, 0], [1, 0, 0],
                  [0, -1, 0], [0, 0, -1], [0, 0, 0], [0, 0, 0]], dtype=np.float64)
    P = np.zeros((3, 9))
    P[0, 0] = P[1, 1] = P[2, 2] = 1
    D = np.diag([1 / (1 + n * chi), 1 / (1 + m * chi), 1 / (1 + m * chi)])
    S = np.diag(np.asarray(s, dtype=np.float64))
    I9 = np.eye(9)
    if v == 0:
        X = np.zeros((9, 9))
    elif v == 1:
        X = I9
    elif v == 2:
        X = J @ D @ P
    else:
        X = L @ D @ P
    return I9 + S @ (J @ D @ P - I9) - chi * X


def amplification(A, kx, ky):
    """G(k) = diag(exp(-i k.c)) A for arrays of wavenumbers -> (nk, 9, 9)."""
    kx = np.atleast_1d(np.asarray(kx, dtype=np.float64))
    ky = np.atleast_1d(np.asarray(ky, dtype=np.float64))
    ph = np.exp(-1j * (np.outer(kx, CX) + np.outer(ky, CY)))  # (nk, 9)
    return ph[:, :, None] * A[None, :, :]


def sort_eigs(lam):
    """Sort each row of eigenvalues by (-|lambda|, arg lambda)."""
    lam = np.atleast_2d(lam)
    out = np.empty_like(lam)
    for r in range(lam.shape[0]):
        order = np.lexsort((np.angle(lam[r]), -np.abs(lam[r])))
        out[r] = lam[r][order]
    return out


def eigenvalues(s, chi, qref, kx, ky, n=0.5, m=0.5, variant="II"):
    """LAPACK eigenvalues of G(k) for each k -> (nk, 9), sorted."""
    A = linearized_collision(s, chi, qref, n, m, variant)
    G = amplification(A, kx, ky)
    return sort_eigs(np.linalg.eigvals(G))


def bgk(s):
    """BGK as the MRT special case S = s * 1 (eq. eq_BGK_LBM_R)."""
    return (s,) * 9
