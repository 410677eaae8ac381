"""The oracle pins catch plausible mistakes.

Each case plants one mistake (a dropped factor, a flipped sign, a wrong
coefficient) in a private copy of ``oracle/pnref.c``, builds it on the CPU,
and requires at least one of the pins in ``test_oracle_pins.py`` to fail.
"""
import importlib.util
import os
import subprocess

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pnref.c")

# (name, exact text in pnref.c, replacement); each text must occur.
MUTATIONS = [
    ("star_4u_i", "4.0 * u[i] + u[j] - 0.5 * dot3(d, bj);\n      double D",
     "3.0 * u[i] + u[j] - 0.5 * dot3(d, bj);\n      double D"),
    ("star_half_xb_sign", "4.0 * u[i] + u[j] - 0.5 * dot3(d, bj);\n      double D",
     "4.0 * u[i] + u[j] + 0.5 * dot3(d, bj);\n      double D"),
    ("star_D_coeff", "double D = 4.0 * dot3(n, vi) - 3.0 * nvj;\n      for (int q = 0; q < 3; ++q)\n        out[q] += k * (S * n[q] + D * (vi[q] - vj[q])) - 3.5 * (G * mass[j] / R) * bj[q];\n    }\n    acc_1pn",
     "double D = 4.0 * dot3(n, vi) - 2.0 * nvj;\n      for (int q = 0; q < 3; ++q)\n        out[q] += k * (S * n[q] + D * (vi[q] - vj[q])) - 3.5 * (G * mass[j] / R) * bj[q];\n    }\n    acc_1pn"),
    ("star_7half_b", "D * (vi[q] - vj[q])) - 3.5 * (G * mass[j] / R) * bj[q];\n    }\n    acc_1pn",
     "D * (vi[q] - vj[q])) - 2.5 * (G * mass[j] / R) * bj[q];\n    }\n    acc_1pn"),
    ("bh_pair_V0", "double br = -vi2 + 4.0 * dot3(vi, w) + 4.0 * Vi + V0 + 0.5 * dot3(d, aN0);\n      double n4v",
     "double br = -vi2 + 4.0 * dot3(vi, w) + 4.0 * Vi - V0 + 0.5 * dot3(d, aN0);\n      double n4v"),
    ("bh_pair_w_sign", "n4v * (vi[q] - w[q]) - 3.0 * nw * vi[q]) +\n                  3.5 * (G * M / R) * aN0[q];\n    }\n    /* partners",
     "n4v * (vi[q] + w[q]) - 3.0 * nw * vi[q]) +\n                  3.5 * (G * M / R) * aN0[q];\n    }\n    /* partners"),
    ("bh_pair_7half", "- 3.0 * nw * vi[q]) +\n                  3.5 * (G * M / R) * aN0[q];\n    }\n    /* partners",
     "- 3.0 * nw * vi[q]) +\n                  2.5 * (G * M / R) * aN0[q];\n    }\n    /* partners"),
    ("w_sign", "const double w[3] = {-P[0] / M, -P[1] / M, -P[2] / M};\n  const double V0 = -phi[0];",
     "const double w[3] = {P[0] / M, P[1] / M, P[2] / M};\n  const double V0 = -phi[0];"),
    ("bh_4V0", "1.5 * nvs * nvs + 4.0 * V0 +\n                  Vs + 0.5 * dot3(d, aNs);\n      double nw = dot3(n, w);\n      for (int q = 0; q < 3; ++q)\n        out[q] += k * (br * n[q] + 3.0 * nvs * vs[q] - 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +\n                  3.5 * (G * mass[s] / R) * aNs[q];\n    }\n    acc_1pn[0]",
     "1.5 * nvs * nvs + 3.0 * V0 +\n                  Vs + 0.5 * dot3(d, aNs);\n      double nw = dot3(n, w);\n      for (int q = 0; q < 3; ++q)\n        out[q] += k * (br * n[q] + 3.0 * nvs * vs[q] - 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +\n                  3.5 * (G * mass[s] / R) * aNs[q];\n    }\n    acc_1pn[0]"),
    ("bh_nw_sign", "- 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +\n                  3.5 * (G * mass[s] / R) * aNs[q];\n    }\n    acc_1pn[0]",
     "- 3.0 * nvs * w[q] + 4.0 * nw * vs[q]) +\n                  3.5 * (G * mass[s] / R) * aNs[q];\n    }\n    acc_1pn[0]"),
    ("bh_vs2", "double br = -2.0 * dot3(vs, vs) + 4.0 * dot3(w, vs) + 1.5 * nvs * nvs + 4.0 * V0 +\n                  Vs + 0.5 * dot3(d, aNs);\n      double nw = dot3(n, w);\n      for (int q = 0; q < 3; ++q)\n        out[q] += k * (br * n[q] + 3.0 * nvs * vs[q] - 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +\n                  3.5 * (G * mass[s] / R) * aNs[q];\n    }\n    acc_1pn[0]",
     "double br = -1.0 * dot3(vs, vs) + 4.0 * dot3(w, vs) + 1.5 * nvs * nvs + 4.0 * V0 +\n                  Vs + 0.5 * dot3(d, aNs);\n      double nw = dot3(n, w);\n      for (int q = 0; q < 3; ++q)\n        out[q] += k * (br * n[q] + 3.0 * nvs * vs[q] - 3.0 * nvs * w[q] - 4.0 * nw * vs[q]) +\n                  3.5 * (G * mass[s] / R) * aNs[q];\n    }\n    acc_1pn[0]"),
    ("energy_bh_v2", "E1 += 1.5 * G * M * mass[i] / r1i * vi2;", "E1 += 2.5 * G * M * mass[i] / r1i * vi2;"),
    ("energy_pair_7", "E1 += 0.25 * k * (6.0 * vi2 - 7.0 * dot3(vi, vj)",
     "E1 += 0.25 * k * (6.0 * vi2 - 6.0 * dot3(vi, vj)"),
    ("energy_i_eq_j", "E1 += 0.5 * M * sum_over_r1i * sum_over_r1i;",
     "E1 += 0.25 * M * sum_over_r1i * sum_over_r1i;"),
    ("momentum_nn_sign", "P1[q] -= 0.5 * k * (vi[q] + vin2 * nij[q]);",
     "P1[q] -= 0.5 * k * (vi[q] - vin2 * nij[q]);"),
    ("newton_softening", "return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2);",
     "return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 2.0 * eps2);"),
    ("rk4_weight", "pos[t] += dt / 6.0 * (kx1[t] + 2.0 * kx2[t] + 2.0 * kx3[t] + kx4[t]);",
     "pos[t] += dt / 6.0 * (kx1[t] + 2.0 * kx2[t] + 1.0 * kx3[t] + 2.0 * kx4[t]);"),
    ("jerk_richardson_weight", "const double w = (k == 1) ? 8.0 : -1.0;",
     "const double w = (k == 1) ? 7.0 : -1.0;"),
    ("jerk_no_velocity_shift", "vs[t] = vel[t] + hh * acc_out[t];", "vs[t] = vel[t];"),
    ("hermite_corrector_jerk", "dt2 / 12.0 * (j[t] - jp[t]);", "dt2 / 10.0 * (j[t] - jp[t]);"),
    ("hermite_position_corrector_sign", "dt2 / 12.0 * (a[t] - ap[t]);\n      vel[t] = vn;",
     "dt2 / 12.0 * (ap[t] - a[t]);\n      vel[t] = vn;"),
    ("hermite_velocity_predictor_without_snap",
     "vp[t] = vel[t] + dt * a[t] + dt2 / 2.0 * j[t] + dt3 / 6.0 * sn[t] + dt4 / 24.0 * cr[t];",
     "vp[t] = vel[t] + dt * a[t] + dt2 / 2.0 * j[t];"),
    ("hermite_crackle_sign", "+ 6.0 * dt * (j[t] + jp[t])) / dt3;",
     "- 6.0 * dt * (j[t] + jp[t])) / dt3;"),
    ("jerk_exact_velocity_direction_newtonian_only",
     "W[t] = vel[t] + I * (h * (raN[t] + ra1[t]));", "W[t] = vel[t] + I * (h * raN[t]);"),
    ("jerk_exact_no_position_direction", "X[t] = pos[t] + I * (h * vel[t]);", "X[t] = pos[t];"),
    ("jerk_exact_w_from_unperturbed_velocities",
     "for (int q = 0; q < 3; ++q) w[q] += mass[s] * W[3 * s + q];",
     "for (int q = 0; q < 3; ++q) w[q] += mass[s] * vel[3 * s + q];"),
    ("jerk_exact_star_half_xb_sign", "u[j] - 0.5 * cdot3(d, bj);", "u[j] + 0.5 * cdot3(d, bj);"),
    ("jerk_exact_bh_Vs_sign", "4.0 * V0 + V[s] +", "4.0 * V0 - V[s] +"),
    ("eih_row_Vb_sign", "4.0 * Va - phi[b] + 0.5 * dot3(xab, aNb);",
     "4.0 * Va + phi[b] + 0.5 * dot3(xab, aNb);"),
    ("eih_row_velocity_difference", "k * D * (va[q] - vb[q]) + 3.5 * (G * mass[b] / R) * aNb[q];\n  }\n}",
     "k * D * (va[q] + vb[q]) + 3.5 * (G * mass[b] / R) * aNb[q];\n  }\n}"),
    ("jerk_exact_b_of_unperturbed_position",
     "for (int q = 0; q < 3; ++q) b[3 * s + q] = G * M * d[q] / (R * R * R);",
     "for (int q = 0; q < 3; ++q) b[3 * s + q] = G * M * creal(d[q]) / (R * R * R);"),
]

# the pins run against each mutant (the mutation test must not rely on P6's
# long integration alone; every mutant is caught by one of these)
PIN_CALLS = [
    lambda m: pins.test_p3_two_body_limit(m),
    lambda m: pins.test_p3_test_particle_is_schwarzschild_harmonic(m),
    lambda m: pins.test_p3_hand_reduced_two_body_fixture(m),
    lambda m: pins.test_p2_truncation_order_against_full_eih(m),
    lambda m: [pins.test_p1_literal_equations_match_eih_layout(m, s, 10.0) for s in (0, 1)],
    lambda m: pins.test_energy_momentum_two_body_textbook(m),
    lambda m: pins.test_p7_energy_conserved_at_1pn(m),
    lambda m: pins.test_p6_periapsis_advance(m),
    lambda m: pins.test_softening_changes_cross_terms_only_at_order_eps2(m),
    lambda m: pins.test_p10_plummer_softening_closed_form(m),
    lambda m: pins.test_jerk_newtonian_closed_form(m),
    lambda m: pins.test_jerk_is_the_time_derivative_along_the_motion(m),
    lambda m: pins.test_hermite_fourth_order_and_precession(m, 2e-5),
    lambda m: pins.test_hermite_fourth_order_with_velocity_dependent_force(m, 3e-5),
    lambda m: pins.test_jerk_exact_value_part_is_the_acceleration(m, 3.0),
    lambda m: pins.test_jerk_exact_newtonian_closed_form(m, 1e-2),
    lambda m: pins.test_jerk_exact_two_body_closed_form(m),
    lambda m: pins.test_difference_quotient_converges_to_exact_jerk_as_h4(m, 3.0),
    lambda m: pins.test_jerk_exact_is_the_time_derivative_along_the_motion(m),
    lambda m: pins.test_hermite_fourth_order_with_velocity_dependent_force(m, 0.0),
    lambda m: pins.test_eih_potentials_once_equals_brute_force(m),
]


def _load_mutant(tmp_path, name, old, new):
    with open(SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation {name}: anchor text must occur exactly once"
    csrc = tmp_path / f"{name}.c"
    csrc.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-std=c11", "-o", str(so), str(csrc), "-lm"])
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}",
                                                  os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB_PATH = str(so)
    return mod


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    mod = _load_mutant(tmp_path, name, old, new)
    for call in PIN_CALLS:
        try:
            call(mod)
        except (AssertionError, ValueError):
            return  # caught
    pytest.fail(f"no pin caught the planted mistake {name}")
