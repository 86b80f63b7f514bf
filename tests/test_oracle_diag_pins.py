"""Pins of the oracle's diagnostics (the monitored sums and the maximum
deviation; Sec. 4.1 tracks E_L2 = sqrt(sum (rho - rho_0)^2 / N)) against
closed forms: the base state, a single planted deviation, a uniform
perturbation, a sine density whose squared sum follows from discrete
orthogonality, and non-finite cells."""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def uniform_state(nx, ny, rho, ux, uy):
    return oracle.feq_field(np.full((ny, nx), rho), np.full((ny, nx), ux), np.full((ny, nx), uy))


def _paper_velocities():
    """Velocities read off rows 1 and 2 of the printed matrix (App. A.1)."""
    M = np.loadtxt(os.path.join(GOLD, "d2q9_M.txt"))
    return M[1].astype(int), M[2].astype(int)


def test_diagnostics_of_the_base_state_vanish():
    """The base state f^eq(rho_b, u_b) with a mean flow has no deviation at
    all: every sum and the maximum deviation are zero (deviations are taken
    from the moving equilibrium, not from w_i rho_b, and momentum deviations
    from rho_b u_b)."""
    rb, ub = 1.02, (0.11, -0.07)
    f = uniform_state(13, 7, rb, *ub)
    d = oracle.diagnostics(f, rb, *ub)
    np.testing.assert_allclose(d, 0.0, rtol=0, atol=1e-15 * f.shape[1] * f.shape[2])


@pytest.mark.parametrize("cell", [(0, 0), (5, 3), (12, 6)])
def test_diagnostics_single_planted_deviation(cell):
    """One population of one cell moved by e from the base state: the sums
    are e, e c_i, e^2 and e^2 |c_i|^2 whatever the cell, the maximum
    deviation is |e|, and no cell is non-finite."""
    rb, ub = 0.97, (0.05, 0.08)
    cxp, cyp = _paper_velocities()
    for i in range(9):
        for e in (3e-4, -2e-3):
            f = uniform_state(13, 7, rb, *ub)
            f[i, cell[1], cell[0]] += e
            d = oracle.diagnostics(f, rb, *ub)
            c2 = cxp[i] ** 2 + cyp[i] ** 2
            expect = [e, e * cxp[i], e * cyp[i], e * e, e * e * c2, abs(e), 0.0]
            np.testing.assert_allclose(d, expect, rtol=1e-9, atol=1e-14)


def test_diagnostics_uniform_perturbation_closed_form():
    """A uniform state f^eq(rho, u) over N cells: sum drho = N (rho - rho_b),
    sum dj = N (rho u - rho_b u_b), and the squares likewise."""
    nx, ny = 11, 6
    N = nx * ny
    rb, ub = 1.0, (0.1, 0.0)
    rho, u = 1.0 + 4e-4, (0.1 - 2e-4, 3e-4)
    f = uniform_state(nx, ny, rho, *u)
    d = oracle.diagnostics(f, rb, *ub)
    dr = rho - rb
    dj = (rho * u[0] - rb * ub[0], rho * u[1] - rb * ub[1])
    np.testing.assert_allclose(d[:5], [N * dr, N * dj[0], N * dj[1], N * dr * dr,
                                       N * (dj[0] ** 2 + dj[1] ** 2)], rtol=1e-9)
    assert d[6] == 0


def test_diagnostics_l2_of_a_sine_density():
    """rho = rho_b + eps sin(2 pi x / nx) at rest: sum drho = 0 and
    sum drho^2 = N eps^2 / 2 (discrete orthogonality), so
    E_L2 = sqrt(sum drho^2 / N) = eps / sqrt(2) (Sec. 4.1)."""
    nx, ny, eps = 24, 5, 1e-3
    x = np.arange(nx)
    rho = np.broadcast_to(1.0 + eps * np.sin(2 * np.pi * x / nx), (ny, nx))
    f = oracle.feq_field(rho, np.zeros((ny, nx)), np.zeros((ny, nx)))
    d = oracle.diagnostics(f, 1.0, 0.0, 0.0)
    assert abs(d[0]) < 1e-15
    np.testing.assert_allclose(np.sqrt(d[3] / (nx * ny)), eps / np.sqrt(2), rtol=1e-10)
    np.testing.assert_allclose(d[1:3], 0.0, atol=1e-16)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_diagnostics_non_finite_cell(bad):
    """A cell with a non-finite population is counted once, makes the sums
    non-finite, and is left out of the maximum deviation, which is taken
    over the finite cells."""
    rb = 1.0
    f = uniform_state(9, 8, rb, 0.0, 0.0)
    f[2, 4, 4] += 7e-4            # the largest deviation among finite cells
    f[5, 1, 6] = bad              # non-finite cell ...
    f[0, 1, 6] += 0.5             # ... whose other populations deviate more
    d = oracle.diagnostics(f, rb, 0.0, 0.0)
    assert d[6] == 1
    assert not np.isfinite(d[0]) and not np.isfinite(d[3])
    np.testing.assert_allclose(d[5], 7e-4, rtol=1e-9)
    g = uniform_state(9, 8, rb, 0.0, 0.0)
    g[:, 2, 2] = np.nan
    g[:, 3, 3] = np.inf
    assert oracle.diagnostics(g, rb, 0.0, 0.0)[6] == 2
    h = np.full((9, 2, 3), np.nan)
    dh = oracle.diagnostics(h, rb, 0.0, 0.0)
    assert dh[6] == 6 and dh[5] == 0.0
