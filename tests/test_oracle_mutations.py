"""The pins must catch a plausible mistake anywhere in the oracle.

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a wrong sign, index, factor or operand), builds it, and runs the fast
pin suite against it with LBMREF_LIB: the suite must fail. The mistakes are
planted on the CPU, in the oracle only.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

MUTANTS = {
    "drop_u2_term": ("4.5 * eu * eu - 1.5 * usq", "4.5 * eu * eu"),
    "wrong_quadratic_coeff": ("4.5 * eu * eu", "3.0 * eu * eu"),
    "source_sign": ("s[i] = 3.0 * w[i] * alpha", "s[i] = -3.0 * w[i] * alpha"),
    "alpha_sign": ("return 1.0 / 3.0 - c2;", "return c2 - 1.0 / 3.0;"),
    "forward_difference_x": ("L->R[(size_t)y * nx + wrap(x - 1, nx)]) / 2.0", "L->R[s]) / 1.0"),
    "missing_half_y": ("L->R[(size_t)wrap(y - 1, ny) * nx + x]) / 2.0", "L->R[(size_t)wrap(y - 1, ny) * nx + x]) / 1.0"),
    "swapped_gradient": ("0.0 : alpha, gx, gy, src)", "0.0 : alpha, gy, gx, src)"),
    "y_gradient_wrong_column": ("L->R[(size_t)wrap(y + 1, ny) * nx + x]", "L->R[(size_t)wrap(y + 1, ny) * nx + wrap(x + 1, nx)]"),
    "stream_backwards_x": ("int xd = wrap(x + e[2 * i], nx);", "int xd = wrap(x - e[2 * i], nx);"),
    "stream_transposed": ("int yd = wrap(y + e[2 * i + 1], ny);", "int yd = wrap(y + e[2 * i], ny);"),
    "relaxation_off": ("(fi - feq[i]) / L->tau", "(fi - feq[i]) / (L->tau + 0.01)"),
    "diagonal_weight": ("w[i] = 1.0 / 36.0;", "w[i] = 1.0 / 35.0;"),
    "link_angle": ("double a = pi * (i - 4.5) / 2.0;", "double a = pi * (i - 5.5) / 2.0;"),
    "momentum_not_velocity": ("L->UX[s] = jx / rho;", "L->UX[s] = jx;"),
    "u_x_for_u_y": ("double eu = e[2 * i] * ux + e[2 * i + 1] * uy;", "double eu = e[2 * i] * ux + e[2 * i + 1] * ux;"),
    # the altered-equilibrium model
    "c2_rest_share": ("feq[0] = rho - moving;", "feq[0] = w[0] * rho;"),
    "c2_ignored": ("w[i] * rho * (3.0 * c2 + 3.0 * eu", "w[i] * rho * (1.0 + 3.0 * eu"),
    "c2_model_keeps_source": ("L->model == LBMREF_MODEL_EQUILIBRIUM ? 0.0 : alpha", "alpha"),
    # a c2 field (alpha varying in space)
    "c2_field_ignored": ("double alpha = L->A ? L->A[s] : L->alpha;", "double alpha = L->alpha;"),
    "c2_field_transposed": ("L->A ? L->A[s]", "L->A ? L->A[(size_t)x * ny + y]"),
    "c2_field_neighbour": ("L->A ? L->A[s]", "L->A ? L->A[(size_t)y * nx + wrap(x + 1, nx)]"),
    "c2_field_sign": ("L->A[s] = lbmref_alpha(c2[s]);", "L->A[s] = c2[s] - 1.0 / 3.0;"),
    # Fig. 1 boundaries
    "inlet_phase": ("sin(2.0 * pi * (double)L->t / L->period)", "sin(2.0 * pi * (double)(L->t + 1) / L->period)"),
    "inlet_cosine": ("sin(2.0 * pi * (double)L->t / L->period)", "cos(2.0 * pi * (double)L->t / L->period) - 1.0"),
    "seam_not_cut": ("fstar = crosses ? entered[i] : own[i];", "fstar = own[i];"),
    "boundary_collides": ("if (xbc && (x == 0 || x == nx - 1)) {", "if (xbc && x < 0) {"),
    "outlet_at_inlet_density": ("model_equilibrium(L, 1.0, 0.0, 0.0, fout);", "model_equilibrium(L, rho_in, 0.0, 0.0, fout);"),
    # compensated totals
    "totals_compensation_dropped": ("double v = sum[k] + comp[k];", "double v = sum[k];"),
    "totals_compensation_sign_small_term": ("*comp += (*sum - t) + v;", "*comp -= (*sum - t) + v;"),
    "totals_compensation_sign_large_term": ("*comp += (v - t) + *sum;", "*comp -= (v - t) + *sum;"),
    "totals_compensation_branch_swapped": ("if (fabs(*sum) >= fabs(v))", "if (fabs(*sum) < fabs(v))"),
}

FAST_PINS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
             os.path.join(ROOT, "tests", "test_oracle_physics.py"),
             os.path.join(ROOT, "tests", "test_oracle_equilibrium_model.py"),
             os.path.join(ROOT, "tests", "test_oracle_c2_field.py"),
             os.path.join(ROOT, "tests", "test_oracle_inlet.py")]


def run_pins_against(source_text, tmp_path):
    (tmp_path / "lbmref.c").write_text(source_text)
    shutil.copy(os.path.join(ORACLE, "lbmref.h"), tmp_path / "lbmref.h")
    lib = tmp_path / "liblbmref.so"
    subprocess.run(["make", "-s", "-C", ORACLE, f"SRC={tmp_path / 'lbmref.c'}", f"OUT={lib}"],
                   check=True, capture_output=True)
    env = dict(os.environ, LBMREF_LIB=str(lib), OMP_NUM_THREADS="4")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not slow", "-p", "no:cacheprovider",
                           *FAST_PINS], cwd=ROOT, env=env, capture_output=True, text=True)


def test_unmutated_copy_passes(tmp_path):
    """Control: the harness itself does not make the pins fail."""
    r = run_pins_against(open(os.path.join(ORACLE, "lbmref.c")).read(), tmp_path)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ORACLE, "lbmref.c")).read()
    assert src.count(old) >= 1, f"mutation target for {name} not found"
    r = run_pins_against(src.replace(old, new, 1), tmp_path)
    assert r.returncode == 1, f"pins did not catch mutant {name} (exit {r.returncode}):\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout.splitlines()[-1]
