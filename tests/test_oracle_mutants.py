"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a wrong coefficient, a dropped term, a flipped
sign, a swapped index, a transposed operand) in a private copy of the C
oracle, builds it with gcc and runs the pin suite against it; every mutant
must make at least one pin fail (the short diagnostics pins run first, then
the main pin suite, stopping at the first failure). Nothing here touches the
GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")

MUTANTS = {
    "feq_quadratic_coefficient": ("4.5 * cj * cj / rho", "4.0 * cj * cj / rho"),
    "feq_drops_u2_term": ("-\n                     1.5 * (jx * jx + jy * jy) / rho", "-\n                     0.0 * (jx * jx + jy * jy) / rho"),
    "flin_wrong_factor": ("W[i] * (rho + 3.0 * (CX[i] * jx", "W[i] * (rho + 2.0 * (CX[i] * jx"),
    "shift_n_for_m": ("(jx + m * chi * jxf) / (1.0 + m * chi)", "(jx + n * chi * jxf) / (1.0 + n * chi)"),
    "shift_denominator": ("(rho + n * chi * rf) / (1.0 + n * chi)", "(rho + n * chi * rf) / (1.0 + chi)"),
    "shift_transposed_component": ("(jy + m * chi * jyf)", "(jy + m * chi * jxf)"),
    "type_II_sign": ("d[k] = chi * (tmp2[k] - meqs[k]);", "d[k] = chi * (meqs[k] - tmp2[k]);"),
    "type_I_uses_meq": ("d[k] = chi * (tmp2[k] - mom[k]);", "d[k] = chi * (tmp2[k] - meqs[k]);"),
    "type_III_unshifted": ("flin(rhos, jxs, jys, tmp);", "flin(rho, jx, jy, tmp);"),
    "type_III_full_eq": ("flin(rf, jxf, jyf, tmp);\n      matvec(M_D2Q9, tmp, a);\n      flin(rhos", "feq(rf, jxf, jyf, tmp);\n      matvec(M_D2Q9, tmp, a);\n      flin(rhos"),
    "relax_sign": ("mom[k] + sk[k] * (meqs[k] - mom[k]) + d[k]", "mom[k] + sk[k] * (mom[k] - meqs[k]) + d[k]"),
    "relax_drops_damping": ("mom[k] + sk[k] * (meqs[k] - mom[k]) + d[k]", "mom[k] + sk[k] * (meqs[k] - mom[k])"),
    "stream_push_direction": ("wrap(x - CX[i], nx), ys = wrap(y - CY[i], ny)", "wrap(x + CX[i], nx), ys = wrap(y + CY[i], ny)"),
    "stream_axes_swapped": ("wrap(x - CX[i], nx), ys = wrap(y - CY[i], ny)", "wrap(x - CY[i], nx), ys = wrap(y - CX[i], ny)"),
    "matvec_transposed": ("acc += A[i][j] * x[j];", "acc += A[j][i] * x[j];"),
    "matrix_entry": ("{ 4, -2, -2, -2, -2, 1,  1,  1,  1}", "{ 4, -2, -2, -2, -2, 1,  1,  1,  2}"),
    "weights_swapped": ("static const double W[Q] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,\n                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};",
                        "static const double W[Q] = {4.0 / 9,  1.0 / 36,  1.0 / 9,  1.0 / 9, 1.0 / 9,\n                            1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36};"),
    "velocity_from_wrong_row": ("CY[j] = (int)M_D2Q9[2][j];", "CY[j] = (int)M_D2Q9[6][j] / -2;"),
    "none_keeps_shift": ("if (variant == V_NONE || variant == V_VISC) chi = 0.0;", "if (variant == V_VISC) chi = 0.0;"),
    "visc_ramp_wrong_end": ("sk[k] = s[k] + (1.0 - s[k]) * xi;", "sk[k] = s[k] + (2.0 - s[k]) * xi;"),
    "mean_from_post_collision": ("matvec(M_D2Q9, fin, mom);  /* pre-collision", "matvec(M_D2Q9, fo, mom);  /* pre-collision"),
    "mean_rate_complement": ("cf[c] = rf + alpha * (mom[0] - rf);", "cf[c] = rf + (1.0 - alpha) * (mom[0] - rf);"),
    "mean_momentum_component": ("cf[2 * N + c] = jyf + alpha * (mom[2] - jyf);", "cf[2 * N + c] = jyf + alpha * (mom[1] - jyf);"),
    "mean_velocity_not_momentum": ("rf, jxf / rf, jyf / rf, s, n, m, variant, fo);", "rf, jxf, jyf, s, n, m, variant, fo);"),
    "source_time_offset": ("const double tn = (double)(t0 + t + 1);", "const double tn = (double)(t0 + t);"),
    "source_velocity_dropped": ("feq(rs, rs * src[4], rs * src[5], fs);", "feq(rs, 0.0, 0.0, fs);"),
    "source_sine_sign": ("src[0] + src[1] * sin(", "src[0] - src[1] * sin("),
    "outflow_wrong_column": ("post[i * N + y * nx + nx - 1] = post[i * N + y * nx + nx - 2];", "post[i * N + y * nx + nx - 1] = post[i * N + y * nx + nx - 3];"),
    "diag_base_without_velocity": ("feq(rho_b, rho_b * ux_b, rho_b * uy_b, fb);", "feq(rho_b, 0.0, 0.0, fb);"),
    "diag_max_over_f": ("const double d = fabs(v - fb[i]);", "const double d = fabs(v);"),
    "diag_jx_from_cy": ("      jx += CX[i] * v;", "      jx += CY[i] * v;"),
    "diag_momentum_base_velocity": ("djx = jx - rho_b * ux_b", "djx = jx - ux_b"),
    "diag_abs_not_square": ("s_r2 += dr * dr;", "s_r2 += fabs(dr);"),
    "diag_max_includes_non_finite": ("    if (finite) {\n      if (dmax > mx) mx = dmax;",
                                     "    if (dmax > mx) mx = dmax;\n    if (finite) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-std=c99", "-o", str(so), str(mut), "-lm"])
    env = dict(os.environ, LBM_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_diag_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])
