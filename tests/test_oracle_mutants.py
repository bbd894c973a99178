"""The oracle's pins catch plausible mistakes.

Each case plants one slip in a copy of the oracle's C source (a sign, a
dropped term, a transposed operand, an unsplit tie, a wrong coefficient),
builds it into a temporary library, and runs the pin suite against it in a
subprocess: every mutant must fail at least one pin.  The real oracle is
never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "zm_oracle.c")

MUTANTS = {
    "bs_sign": ("const double coef = -(h1 * h2) / (4.0 * M_PI);",
                "const double coef = (h1 * h2) / (4.0 * M_PI);"),
    "bs_two_pi": ("const double coef = -(h1 * h2) / (4.0 * M_PI);",
                  "const double coef = -(h1 * h2) / (2.0 * M_PI);"),
    "r3_dropped": ("double r3 = zi3 - zj3;", "double r3 = 0.0 * (zi3 - zj3);"),
    "cross_transposed": ("double x2 = r3 * g1 - r1 * g3;", "double x2 = r1 * g3 - r3 * g1;"),
    "strength_transposed": ("double g1 = w1 * b1 - w2 * a1;\n        double g2 = w1 * b2 - w2 * a2;\n"
                            "        double g3 = w1 * b3 - w2 * a3;",
                            "double g1 = w1 * a1 - w2 * b1;\n        double g2 = w1 * a2 - w2 * b2;\n"
                            "        double g3 = w1 * a3 - w2 * b3;"),
    "image_shift_sign": ("double r1 = zi1 - zj1 - S1 * L1;", "double r1 = zi1 - zj1 + S1 * L1;"),
    "tie_unsplit": ("    weight[0] = 0.5;\n    weight[1] = 0.5;\n    return 2;",
                    "    weight[0] = 1.0;\n    weight[1] = 0.0;\n    return 1;"),
    "eps_not_squared": ("const double eps2 = P->eps * P->eps;", "const double eps2 = P->eps;"),
    "kernel_power": ("double wgt = inv * inv * inv;", "double wgt = inv * inv;"),
    "fd_coefficient": ("return (8.0 * (fp1 - fm1) - (fp2 - fm2)) / (12.0 * h);",
                       "return (8.0 * (fp1 - fm1) - 2.0 * (fp2 - fm2)) / (12.0 * h);"),
    "fd_no_unwrap": ("if (c == 0 && w1 != 0) v = v + (double)w1 * P->period1;", ""),
    "laplacian_coefficient": ("return (-fp2 + 16.0 * fp1 - 30.0 * f0 + 16.0 * fm1 - fm2) / (12.0 * h * h);",
                              "return (-fp2 + 16.0 * fp1 - 32.0 * f0 + 16.0 * fm1 - fm2) / (12.0 * h * h);"),
    "q_no_metric": ("q[p] = (g1 * g1 + g2 * g2 + g3 * g3) / (n1 * n1 + n2 * n2 + n3 * n3);",
                    "q[p] = (g1 * g1 + g2 * g2 + g3 * g3);"),
    "v_q_coefficient": ("return P->atwood * ((uu - 0.25 * q) - (2.0 * P->gravity) * z3);",
                        "return P->atwood * ((uu - 0.5 * q) - (2.0 * P->gravity) * z3);"),
    "v_velocity_squared_dropped": ("double uu = u1 * u1 + u2 * u2 + u3 * u3;",
                                   "double uu = 0.0 * (u1 * u1 + u2 * u2 + u3 * u3);"),
    "gravity_sign": ("return P->atwood * ((uu - 0.25 * q) - (2.0 * P->gravity) * z3);",
                     "return P->atwood * ((uu - 0.25 * q) + (2.0 * P->gravity) * z3);"),
    "rk3_stage2_weights": ("y2[k] = 0.75 * y0[k] + 0.25 * (y1[k] + dt * F[k]);",
                           "y2[k] = 0.25 * y0[k] + 0.75 * (y1[k] + dt * F[k]);"),
    "cutoff_no_image": ("const double r1 = d1 - S1 * L1;", "const double r1 = d1;"),
    "cutoff_eps_changed": ("const double inv = 1.0 / sqrt(dd + eps_sq);",
                           "const double inv = 1.0 / sqrt(dd + 0.25 * eps_sq);"),
    "cutoff_radius_not_squared": ("const double rc2 = P->cutoff * P->cutoff;",
                                  "const double rc2 = P->cutoff;"),
    "cutoff_boundary_inclusive": ("if (!(dd < rc2)) continue;", "if (!(dd <= rc2)) continue;"),
    "low_half_dropped": ("const double f = 0.5 * (c1 * w[pj] + c2 * w[N + pj]);",
                         "const double f = (c1 * w[pj] + c2 * w[N + pj]);"),
    "low_symbol_sign": ("c1 = nyq1 ? 0.0 : k1 / kk;", "c1 = nyq1 ? 0.0 : -k1 / kk;"),
    "low_symbol_power": ("const double kk = sqrt(k1 * k1 + k2 * k2);",
                         "const double kk = (k1 * k1 + k2 * k2);"),
    "low_normal_component": ("u[N + p] = S[p] * (ny * inv);", "u[N + p] = S[p] * (nx * inv);"),
    "free_ghost_quadratic": ("return i == -1 ? 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - g3",
                             "return i == -1 ? 3.0 * g0 - 3.0 * g1 + 1.0 * g2 - 0.0 * g3"),
    "free_far_ghost": ("    return i == n ? 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - g3",
                       "    return i == n ? 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - 2.0 * g3"),
    "free_images_kept": ("int k1 = axis_images(i1, j1, P->boundary == 1 ? -n1 : n1, s1, c1);",
                         "int k1 = axis_images(i1, j1, n1, s1, c1);"),
    "free_cutoff_images_kept": ("const double S1 = free_sheet ? 0.0 : nearbyint(d1 / L1);",
                                "const double S1 = nearbyint(d1 / L1);"),
    "medium_v_from_br": ("        uv = ulo;", "        uv = zt;"),
    "rk3_stage3_weights": ("double y3 = (1.0 / 3.0) * y0[k] + (2.0 / 3.0) * (y2[k] + dt * F[k]);",
                           "double y3 = (1.0 / 2.0) * y0[k] + (1.0 / 2.0) * (y2[k] + dt * F[k]);"),
}


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                    "-shared", str(src), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, ZMO_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_cutoff.py"),
                        os.path.join(ROOT, "tests", "test_oracle_loworder.py"),
                        os.path.join(ROOT, "tests", "test_oracle_free.py"),
                        os.path.join(ROOT, "tests", "test_oracle_medium.py"),
                        os.path.join(ROOT, "tests", "test_oracle_vterms.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
