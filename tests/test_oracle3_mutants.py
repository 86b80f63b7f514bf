"""The D3Q15 oracle's pins must catch plausible mistakes: each case plants one
in a private copy of lbm3_oracle.c, builds it with gcc and runs
tests/test_oracle3_pins.py against it. Nothing here touches the GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm3_oracle.c")

MUTANTS = {
    "matrix_entry": ("{16, -4, -4, -4, -4, -4, -4, 1,  1,  1,  1,  1,  1,  1,  1}",
                     "{16, -4, -4, -4, -4, -4, -4, 1,  1,  1,  1,  1,  1,  1,  2}"),
    "weight_diagonal": ("1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,", "1.0 / 9,  1.0 / 64, 1.0 / 72, 1.0 / 72,"),
    "feq_quadratic": ("4.5 * cj * cj / rho", "4.0 * cj * cj / rho"),
    "velocity_z_from_wrong_row": ("C3Z[j] = (int)M3[3][j];", "C3Z[j] = (int)M3[2][j];"),
    "shift_n_for_m": ("(jz + m * chi * jfz) / (1.0 + m * chi)", "(jz + n * chi * jfz) / (1.0 + n * chi)"),
    "type_II_sign": ("d[k] = chi * (a[k] - (variant == V3_I ? mom[k] : meq[k]));",
                     "d[k] = chi * ((variant == V3_I ? mom[k] : meq[k]) - a[k]);"),
    "type_III_unshifted": ("flin3(rs, jsx, jsy, jsz, tmp);", "flin3(rho, jx, jy, jz, tmp);"),
    "stream_z_push": ("zs = wrap3(z - C3Z[i], nz);", "zs = wrap3(z + C3Z[i], nz);"),
    "relax_sign": ("mom[k] + sk[k] * (meq[k] - mom[k]) + d[k]", "mom[k] + sk[k] * (mom[k] - meq[k]) + d[k]"),
    "visc_ramp_wrong_end": ("sk[k] = s[k] + (1.0 - s[k]) * xi;", "sk[k] = s[k] + (2.0 - s[k]) * xi;"),
    "visc_ramp_squared": ("sk[k] = s[k] + (1.0 - s[k]) * xi;", "sk[k] = s[k] + (1.0 - s[k]) * xi * xi;"),
    "visc_keeps_shift": ("if (variant == V3_NONE || variant == V3_VISC) chi = 0.0;",
                         "if (variant == V3_NONE) chi = 0.0;"),
    "visc_ramp_read_after_zeroing": ("  const double xi = chi;\n  if (variant == V3_NONE || variant == V3_VISC) chi = 0.0;",
                                     "  if (variant == V3_NONE || variant == V3_VISC) chi = 0.0;\n  const double xi = chi;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mut = tmp_path / "mutant3.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "mutant3.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-std=c99", "-o", str(so), str(mut), "-lm"])
    env = dict(os.environ, LBM_ORACLE3_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle3_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])
