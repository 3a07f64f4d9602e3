"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a flipped sign, a transposed operand, a dropped
term, a wrong index) in a temporary copy of oracle.c, builds it on the CPU and
runs the pin suite against that build in a subprocess; the suite must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "rotation_jacobian_sign": ("dX[6 * a + k] = (k < 3) ? (a == k ? 1.0 : 0.0) : -S[3 * a + (k - 3)];",
                               "dX[6 * a + k] = (k < 3) ? (a == k ? 1.0 : 0.0) : S[3 * a + (k - 3)];"),
    "projection_derivative": ("-L->fx * X[0] / (X[2] * X[2])", "-L->fx * X[0] / X[2]"),
    "bilinear_du_weight": ("du[c] = (1.0 - ay) * (f10[c] - f00[c]) + ay * (f11[c] - f01[c]);",
                           "du[c] = (1.0 - ax) * (f10[c] - f00[c]) + ax * (f11[c] - f01[c]);"),
    "gravity_residual_sign": ("r[i] = gc[i] - f->g_imu[i];", "r[i] = gc[i] + f->g_imu[i];"),
    "range_point_transposed": ("mat3T_vec(T, qt, P);", "mat3_vec(T, qt, P);"),
    "range_jacobian_transposed": ("((k < 3) ? -T[3 * k + a] :", "((k < 3) ? -T[3 * a + k] :"),
    "cauchy_weight": ("*drho = 1.0 / (1.0 + s / b);", "*drho = 1.0 / (1.0 + s);"),
    "hessian_drops_weight": ("H[6 * a + b] += W * sum;\n            }\n            double sg = 0.0;\n            for (int k = 0; k < C; ++k)",
                             "H[6 * a + b] += sum;\n            }\n            double sg = 0.0;\n            for (int k = 0; k < C; ++k)"),
    "se3_V_coefficient": ("V[i] = I + B * W[i] + Cp * W2[i];", "V[i] = I + B * W[i] + B * W2[i];"),
    "cholesky_backsub_index": ("s -= L[6 * k + i] * x[k];", "s -= L[6 * i + k] * x[k];"),
    "out_of_view_penalty": ("2.0 * wr, &rho, &drho", "wr, &rho, &drho"),
    "lm_damping_direction": ("lam = lam / f->down;", "lam = lam * f->down;"),
    "acceptance_rule": ("if (cc < c) {\n            if (tr) tr[3] = 1;", "if (cc < c + 1e-3 * fabs(c)) {\n            if (tr) tr[3] = 1;"),
    "pruning_rank_direction": ("if (st[j].c < st[i].c || (st[j].c == st[i].c && j < i)) better++;",
                               "if (st[j].c > st[i].c || (st[j].c == st[i].c && j < i)) better++;"),
    "selection_tie": ("if (best < 0 || cost[m] < cost[best]) best = m;",
                      "if (best < 0 || cost[m] <= cost[best]) best = m;"),
    "gravity_prior_weight": ("c += a_grav * rho;", "c += rho;"),
    "gate_not_squared": ("alpha[s] *= (gate[s] / rn) * (gate[s] / rn);", "alpha[s] *= (gate[s] / rn);"),
    "ratio_cap_direction": ("lam[s] * gn > f->alpha_ratio * gv", "lam[s] * gn < f->alpha_ratio * gv"),
    "cost_tolerance_ignored": ("const int flat = f->cost_tol > 0.0 && fabs(cc - c) <= f->cost_tol * c;",
                               "const int flat = 0;"),
    "cost_tolerance_absolute": ("const int flat = f->cost_tol > 0.0 && fabs(cc - c) <= f->cost_tol * c;",
                                "const int flat = f->cost_tol > 0.0 && fabs(cc - c) <= f->cost_tol;"),
    "qconf_uv_transposed": ("orc_bilinear(L->qconf, L->H, L->W, 1, u, v, &q, &qu, &qv);",
                            "orc_bilinear(L->qconf, L->H, L->W, 1, v, u, &q, &qu, &qv);"),
    "qconf_dropped": ("wq = q;", "wq = 1.0;"),
    "weight_outside_rho": ("        s *= w;\n        orc_robust(L->loss_kind, L->loss_scale, s, &rho, &drho);\n        c += rho;",
                           "        orc_robust(L->loss_kind, L->loss_scale, s, &rho, &drho);\n        c += w * rho;"),
    "scales_from_candidate_gradient": ("orc_prior_scales(f, st->T, g, st->alpha);",
                                       "orc_prior_scales(f, st->T, H, st->alpha);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutated = tmp_path / "oracle.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "oracle.h").write_text(open(os.path.join(ROOT, "oracle", "oracle.h")).read())
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
                           str(mutated), "-o", str(so), "-lm"])
    env = dict(os.environ, PILOT_ORACLE_LIB_OVERRIDE=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
