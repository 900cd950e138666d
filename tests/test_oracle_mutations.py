"""Plant plausible mistakes in a copy of the CPU oracle and check that the pin suite catches
every one of them (a dropped term, a wrong sign, a wrong index or bound, a transposed
operand, a skipped rebuild, a broken wrap). Each mutant is compiled into a temporary
directory with gcc and the pin tests are re-run against it in a child process; the mistake
lives only in that temporary copy, on the CPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle_md.c")
PIN_TESTS = ["tests/test_oracle_invariants.py", "tests/test_oracle_vs_brute.py",
             "tests/test_six_particle.py", "tests/test_oracle_nvt.py",
             "tests/test_oracle_styles.py", "tests/test_oracle_shift.py"]

MUTANTS = {
    "drop_energy_shift": ("lj_energy(s->eps[k], s->sig[k], r2) -\n                lj_energy(",
                          "lj_energy(s->eps[k], s->sig[k], r2) -\n                0.0 * lj_energy("),
    "force_sign_on_i": ("s->f[3 * i + a] += ff * rij[a];", "s->f[3 * i + a] -= ff * rij[a];"),
    "min_image_wrong_sign": ("if (d < -h) return d + L;", "if (d < -h) return d - L;"),
    "list_without_skin": ("double rl = s->rc[k] + s->skin;", "double rl = s->rc[k];"),
    "list_double_counts": ("if (j <= i) continue;", "if (j == i) continue;"),
    "stencil_not_deduplicated": ("if (!seen) stencil[ns++] = e;", "stencil[ns++] = e; (void)seen;"),
    "virial_transposed_index": ("rij[1] * ff * rij[2], rij[2] * ff * rij[2]",
                                "rij[0] * ff * rij[2], rij[2] * ff * rij[2]"),
    "full_kick_instead_of_half": ("double h = 0.5 * s->dt;", "double h = s->dt;"),
    "never_rebuild": ("double lim = 0.5 * s->skin;", "double lim = 50.0 * s->skin;"),
    "wrap_image_sign": ("*x -= L;\n        *img += 1;", "*x -= L;\n        *img -= 1;"),
    "r2_drops_z": ("return t + zz;", "return t + 0.0 * zz;"),
    "force_factor_exponent": ("24.0 * eps * (2.0 * sr12 - sr6) / r2", "24.0 * eps * (2.0 * sr12 - sr6)"),
    # NVT thermostat
    "nvt_first_xi_update_half_step": ("s->xi += 0.25 * s->dt * (2.0 * K - g) * s->invQ;\n    s->eta",
                                      "s->xi += 0.5 * s->dt * (2.0 * K - g) * s->invQ;\n    s->eta"),
    "nvt_eta_full_step": ("s->eta += 0.5 * s->dt * s->xi;", "s->eta += s->dt * s->xi;"),
    "nvt_scale_full_step": ("exp(-0.5 * s->dt * s->xi)", "exp(-s->dt * s->xi)"),
    "nvt_kinetic_not_rescaled": ("K = sc * sc * K;", "K = sc * K;"),
    "nvt_dof_without_momentum": ("return 3.0 * (double)s->n - 3.0;", "return 3.0 * (double)s->n;"),
    # other pair forms
    "mie_prefactor": ("double c = (n / (n - m)) * pow(n / m, m / (n - m));\n        double sr2 = (p[1] * p[1]) / r2;\n        return c * p[0] * (n *",
                      "double c = (m / (n - m)) * pow(n / m, m / (n - m));\n        double sr2 = (p[1] * p[1]) / r2;\n        return c * p[0] * (n *"),
    "gauss_force_missing_width": ("return p[0] / (p[1] * p[1]) * exp(", "return p[0] * exp("),
    "yukawa_force_sign": ("(1.0 + p[1] * r) / (r2 * r)", "(1.0 - p[1] * r) / (r2 * r)"),
    "form_energy_shift_dropped": ("u = form_energy(s->style[k], p, r2) - form_energy(",
                                  "u = form_energy(s->style[k], p, r2) - 0.0 * form_energy("),
    # shifted force
    "shift_force_linear_term_sign": ("u = u + (r - s->rc[k]) * fc;", "u = u - (r - s->rc[k]) * fc;"),
    "shift_force_not_over_r": ("ff = ff - fc / r;", "ff = ff - fc;"),
    "shift_force_cut_force_unscaled": ("double fc = ffc * s->rc[k];", "double fc = ffc;"),
    "nvt_end_half_step_dropped": ("if (s->nvt) thermostat_half(s);\n        s->steps += 1;",
                                  "s->steps += 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(so), str(mut), "-lm"], check=True)
    env = dict(os.environ, LJMD_ORACLE_LIB_OVERRIDE=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_TESTS], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
