"""Sensitivity of the CSPH-TVD oracle's pins: plant plausible slips in a copy
of its C source, build the copy (with the unchanged MUSCL oracle it
includes), and check that tests/test_oracle_csph.py rejects every one.

Planted mistakes live only in temporary copies on the CPU; the committed
oracle is never modified.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "csph_oracle.c")
MUSCL = os.path.join(ROOT, "oracle", "muscl_oracle.c")

# name -> list of (original text, planted text)
MUTATIONS = {
    "pressure_force_sign": [("    Y[1] = -(h * c->phi) * sp + c->rho * g->fx;",
                             "    Y[1] = (h * c->phi) * sp + c->rho * g->fx;")],
    "kernel_normalisation": [("    double g = (2.0 / (3.0 * (h * h))) * f;",
                              "    double g = (1.0 / (h * h)) * f;")],
    "pair_velocity_own_only": [("    double se = a->phi * (0.5 * (c->u + a->u)) * ga",
                                "    double se = a->phi * c->u * ga")],
    "corrector_without_average": [("            AT(Ut, c, j) = 0.5 * (AT(Un, c, j) + AT(Us, c, j)) + hdt * Y[c];",
                                   "            AT(Ut, c, j) = AT(Us, c, j) + hdt * Y[c];")],
    "face_displacement_sign": [("            UL[c] = hl + (0.5 * (h - xt[j + G])) * tl;",
                                "            UL[c] = hl + (0.5 * (h + xt[j + G])) * tl;")],
    "position_update_keeps_predictor": [("        xt[j + G] = 0.5 * xs[j + G] + hdt * (0.5 * (un[j + G] + ut));",
                                         "        xt[j + G] = xs[j + G] + hdt * (0.5 * (un[j + G] + ut));")],
    "predictor_position_end_velocity": [("        xs[j + G] = dt * (0.5 * (un[j + G] + us));",
                                         "        xs[j + G] = dt * us;")],
    "half_step_state_is_old": [("            double hl = 0.5 * (AT(Un, c, j) + AT(Ut, c, j));\n            double hr = 0.5 * (AT(Un, c, j + 1) + AT(Ut, c, j + 1));",
                                "            double hl = AT(Un, c, j);\n            double hr = AT(Un, c, j + 1);")],
    "hll_dissipation_sign": [("            F[c] = (SR * fl - SL * fr + SL * SR * (UR[c] - UL[c])) / (SR - SL);",
                              "            F[c] = (SR * fl - SL * fr - SL * SR * (UR[c] - UL[c])) / (SR - SL);")],
    "relaxation_sign": [("    double s_v = (Ee - c->ev) / tau + c->rho * Q;",
                         "    double s_v = (c->ev - Ee) / tau + c->rho * Q;")],
    "pump_dropped_from_energy": [("    double s_e = c->rho * (c->u * g->fx + Q - I);",
                                  "    double s_e = c->rho * (c->u * g->fx - I);")],
    "distance_displacement_sign": [("    double da = h + (c->xi - a->xi);",
                                    "    double da = h - (c->xi - a->xi);")],
    "slope_not_per_length": [("                                  AT(Un, c, j + 1) - AT(Un, c, j)) / h;",
                              "                                  AT(Un, c, j + 1) - AT(Un, c, j));")],
    "budget_full_step": [("        yE[j + G] = hdt * se;", "        yE[j + G] = dt * se;")],
    "source_ghost_one_cell_off": [("            or_source_ghost(g, gr, t, j, 0, Ug);",
                                   "            or_source_ghost(g, gr, t, j + 1, 0, Ug);")],
    "source_ignores_time": [("            or_source_ghost(g, gr, t, j, 0, Ug);",
                             "            or_source_ghost(g, gr, 0.0, j, 0, Ug);")],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTATIONS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new, 1)
    c = tmp_path / "csph_oracle.c"
    so = tmp_path / "m.so"
    c.write_text(src)
    shutil.copy(MUSCL, tmp_path / "muscl_oracle.c")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-I",
                           str(tmp_path), "-o", str(so), str(c), "-lm"])
    env = dict(os.environ, NG_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_csph.py"),
                        "-q", "-x", "-p", "no:cacheprovider"], env=env, capture_output=True,
                       text=True, cwd=ROOT, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
