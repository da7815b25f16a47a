"""Sensitivity of the oracle's pins: plant plausible slips in a copy of the
oracle's C source (a dropped term, a wrong sign, a wrong index, a wrong
factor), build the copy, and check that the pin suite rejects every one.

Planted mistakes live only in temporary copies on the CPU; the committed
oracle is never modified.
"""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "muscl_oracle.c")

# name -> list of (original text, planted text)
MUTATIONS = {
    "predictor_continuity_drops_rho_du": [
        ("double ax_r = u * sr + rho * su;", "double ax_r = u * sr;"),
        ("ay_r = v * tr + rho * tv;", "ay_r = v * tr;")],
    "predictor_vib_drops_E_du": [
        ("double ax_e = u * se + ev * su;", "double ax_e = u * se;"),
        ("ay_e = v * te + ev * tv;", "ay_e = v * te;")],
    "predictor_momentum_pressure_sign": [
        ("double ax_u = u * su + sp / rho;", "double ax_u = u * su - sp / rho;"),
        ("ay_v = v * tv + tp / rho;", "ay_v = v * tv - tp / rho;")],
    "predictor_pressure_drops_gamma": [
        ("double ax_p = u * sp + gam * p * su;", "double ax_p = u * sp + p * su;"),
        ("ay_p = v * tp + gam * p * tv;", "ay_p = v * tp + p * tv;")],
    "predictor_y_only_sign": [("ay_v = v * tv + tp / rho;", "ay_v = v * tv - tp / rho;")],
    "predictor_drops_sources": [
        ("e_h = ev - hdtdx * ax_e + (dEr + hdt * (rho * Q));", "e_h = ev - hdtdx * ax_e;")],
    "pump_sign_in_energy": [
        ("            Y[3] = rho * (u * g->fx + v * g->fy + Q - I);",
         "            Y[3] = rho * (u * g->fx + v * g->fy - Q - I);")],
    "relaxation_with_rho_factor": [
        ("Y[4] = (Ee - ev) / tau + rho * Q;\n\n            double Un",
         "Y[4] = rho * ((Ee - ev) / tau + Q);\n\n            double Un")],
    "face_state_full_slope": [
        ("WL[c] = Wh[c * ne + m] + 0.5 * Sx[c * ne + m];", "WL[c] = Wh[c * ne + m] + Sx[c * ne + m];")],
    "hllc_star_energy_sign": [
        ("Us[3] = fac * (EL / rL + (Ss - uL) * (Ss + pL / (rL * dL)));",
         "Us[3] = fac * (EL / rL + (Ss - uL) * (Ss - pL / (rL * dL)));")],
    "davis_speed_drops_sound": [
        ("double SR = fmax(uL + cL, uR + cR);", "double SR = fmax(uL + cL, uR);")],
    "y_flux_wrong_neighbour": [
        ("double dG = Gy[c * ne + m] - Gy[c * ne + m - e.nxe];",
         "double dG = Gy[c * ne + m] - Gy[c * ne + m - 1];")],
    "limiter_takes_larger_slope": [
        ("if (a > 0.0 && b > 0.0) return a < b ? a : b;",
         "if (a > 0.0 && b > 0.0) return a > b ? a : b;")],
    "equilibrium_energy_drops_rho": [
        ("double Ee = rho * g->Cv * T;\n            double Y[5];",
         "double Ee = g->Cv * T;\n            double Y[5];")],
    "eq16_drops_factor_two": [
        ("return fmax(vel + c, 2.0 * vel);", "return fmax(vel + c, vel);")],
    "stiff_branch_sign": [
        ("de = ((Ee + tau * (rho * Q)) - Un[4]) * (-expm1(-z));",
         "de = ((Ee + tau * (rho * Q)) - Un[4]) * (expm1(-z));")],
    "stiff_predictor_relaxes_whole_step": [
        ("(-expm1(-(hdt / tau)))", "(-expm1(-(dt / tau)))")],
    "stiff_update_relaxes_from_midstep": [
        ("de = ((Ee + tau * (rho * Q)) - Un[4]) * (-expm1(-z));",
         "de = ((Ee + tau * (rho * Q)) - ev) * (-expm1(-z));")],
    "stiff_update_drops_pump": [
        ("de = ((Ee + tau * (rho * Q)) - Un[4]) * (-expm1(-z));",
         "de = (Ee - Un[4]) * (-expm1(-z));")],
    "stiff_predictor_drops_pump": [
        ("dEv = ((Ee + tau * (rho * Q)) - ev)", "dEv = (Ee - ev)")],
    "stiff_predictor_pressure_drops_sink": [
        ("p_h = p - hdtdx * ax_p - gm1 * (dEv - hdt * (rho * (Q - I)));",
         "p_h = p - hdtdx * ax_p - gm1 * (dEv - hdt * (rho * Q));"),
        ("p_h = p - hdtdx * (ax_p + ay_p) - gm1 * (dEv - hdt * (rho * (Q - I)));",
         "p_h = p - hdtdx * (ax_p + ay_p) - gm1 * (dEv - hdt * (rho * Q));")],
    "tau_wrong_exponent": [
        ("or_pow(T / g->T0, g->tau_T);", "or_pow(T / g->T0, g->tau_rho);")],
    "power_law_half_exponent": [("if (a == 0.5) return sqrt(x);", "if (a == 0.5) return x;")],
    "wall_keeps_normal_momentum": [("            if (fx_) Uc[1] = -Uc[1];\n", "")],
    "wall_mirror_off_by_one": [("return j < 0 ? -1 - j : 2 * n - 1 - j;",
                                "return j < 0 ? -j : 2 * n - 2 - j;")],
    "outflow_copies_wrong_cell": [
        ("if (bc == OR_BC_OUTFLOW || bc == OR_BC_SOURCE) return j < 0 ? 0 : n - 1;",
         "if (bc == OR_BC_OUTFLOW || bc == OR_BC_SOURCE) return j < 0 ? 1 : n - 2;")],
    "source_wave_runs_backwards": [("W[1] = (c / rho_b) * s;", "W[1] = -(c / rho_b) * s;")],
    "source_pressure_not_isentropic": [("W[3] = p_b + (c * c) * s;", "W[3] = p_b + c * s;")],
    "source_ignores_time": [("sin(omega * t - k * x)", "sin(-k * x)")],
    "source_vibrational_energy_fixed": [("W[4] = ev_b + (ev_b / rho_b) * s;", "W[4] = ev_b;")],
    "source_ghost_one_cell_off": [("double x = ((double)j + 0.5) * gr->h;\n    double s =",
                                   "double x = ((double)j + 1.5) * gr->h;\n    double s =")],
    "wedge_inverted": [("return (dx >= 0.0 && fabs(y - gr->wedge_y0) <= dx * gr->wedge_tan) ? 1.0 : 0.0;",
                        "return (dx >= 0.0 && fabs(y - gr->wedge_y0) <= dx * gr->wedge_tan) ? 0.0 : 1.0;")],
    "wedge_leaves_sink_on": [("            double I = act * or_I(g, rho, T);\n            double Ee",
                              "            double I = or_I(g, rho, T);\n            double Ee")],
    "source_segment_ignored": [("    if (!(gr->src_hw > 0.0)) return 1;", "    return 1;")],
    "source_segment_off_by_one_row": [("    double y = ((double)k + 0.5) * gr->h;\n    return fabs",
                                       "    double y = ((double)k + 1.5) * gr->h;\n    return fabs")],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTATIONS[name]:
        assert old in src, (name, old)
        src = src.replace(old, new, 1)
    c = tmp_path / "m.c"
    so = tmp_path / "m.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                           str(so), str(c), "-lm"])
    env = dict(os.environ, NG_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"),
                        "-q", "-x", "-p", "no:cacheprovider"], env=env, capture_output=True,
                       text=True, cwd=ROOT, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
