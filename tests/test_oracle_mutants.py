"""Each plausible slip in the oracle fails at least one of its pins.

Every case copies ``oracle/nb6_oracle.c`` to a temporary directory, plants
one mistake by text substitution, builds it with gcc and runs every pin
against that build.  The clean oracle passes all pins (``test_oracle.py``);
a mutant that passed them all would show a blind spot of the pins.
"""
import os

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "nb6_oracle.c")

MUTANTS = {
    "R_sign": ("R[c] = xp[3 * j + c] - xp[3 * i + c];", "R[c] = xp[3 * i + c] - xp[3 * j + c];"),
    "V_sign": ("V[c] = vp[3 * j + c] - vp[3 * i + c];", "V[c] = vp[3 * i + c] - vp[3 * j + c];"),
    "drop_jerk_rv_term": ("m[j] * (V[c] / r3 - 3.0 * rv * R[c] / r5)", "m[j] * (V[c] / r3)"),
    "jerk_rv_sign": ("m[j] * (V[c] / r3 - 3.0 * rv * R[c] / r5)", "m[j] * (V[c] / r3 + 3.0 * rv * R[c] / r5)"),
    "jerk_factor_2": ("m[j] * (V[c] / r3 - 3.0 * rv * R[c] / r5)", "m[j] * (V[c] / r3 - 2.0 * rv * R[c] / r5)"),
    "r_cubed_as_squared": ("double r3 = r2 * r;\n            double r5", "double r3 = r2;\n            double r5"),
    "r5_as_r4": ("double r5 = r3 * r2;\n            double rv = R[0]", "double r5 = r2 * r2;\n            double rv = R[0]"),
    "mass_of_i": ("nsum_add(&A[c], m[j] * R[c] / r3);", "nsum_add(&A[c], m[i] * R[c] / r3);"),
    "no_velocity_criterion": ("P[c] = R[c] + dti * V[c];", "P[c] = R[c];"),
    "velocity_criterion_backwards": ("P[c] = R[c] + dti * V[c];", "P[c] = R[c] - dti * V[c];"),
    "max_not_min": ("double rmin2 = (p2 < r2) ? p2 : r2;\n\n", "double rmin2 = (p2 < r2) ? r2 : p2;\n\n"),
    "tie_is_neighbour": ("if (rmin2 < hi2) {", "if (rmin2 <= hi2) {"),
    "neighbours_keep_force": ("++count;\n                continue;", "++count;"),
    "self_not_excluded": ("if (j == i) continue;", ""),
    "list_stores_i": ("list[q * lcap + count] = (int32_t)j;", "list[q * lcap + count] = (int32_t)i;"),
    "predict_half_missing": ("a[q] * dt * dt / 2.0\n", "a[q] * dt * dt\n"),
    "predict_jerk_factorial": ("jerk[q] * dt * dt * dt / 6.0", "jerk[q] * dt * dt * dt / 2.0"),
    "predict_velocity_jerk": ("vp[q] = v[q] + a[q] * dt + jerk[q] * dt * dt / 2.0;",
                              "vp[q] = v[q] + a[q] * dt + jerk[q] * dt * dt / 6.0;"),
    "predict_dt_sign": ("double dt = tb - t[k];", "double dt = t[k] - tb;"),
    "uncompensated_drop": ("a->c += (a->s - s) + t;", "a->c += 0.0;"),
    "pair_terms_R_sign": ("R[c] = xp[3 * j + c] - xp[3 * i + c];\n            V[c] = vp[3 * j + c] - vp[3 * i + c];\n            P[c] = R[c] + dtr[p] * V[c];",
                          "R[c] = xp[3 * i + c] - xp[3 * j + c];\n            V[c] = vp[3 * j + c] - vp[3 * i + c];\n            P[c] = R[c] + dtr[p] * V[c];"),
    "pair_terms_jerk_sign": ("djrk[3 * p + c] = m[j] * (V[c] / r3 - 3.0 * rv * R[c] / r5);",
                             "djrk[3 * p + c] = m[j] * (V[c] / r3 + 3.0 * rv * R[c] / r5);"),
    "pair_terms_rmin_max": ("rmin[p] = sqrt((p2 < r2) ? p2 : r2);", "rmin[p] = sqrt((p2 < r2) ? r2 : p2);"),
    # the scale sums every error bar divides by
    "scale_sa_power": ("nsum_add(&SA, m[j] / r2);", "nsum_add(&SA, m[j] / r3);"),
    "scale_sa_mass_of_i": ("nsum_add(&SA, m[j] / r2);", "nsum_add(&SA, m[i] / r2);"),
    "scale_sj_factor": ("nsum_add(&SJ, m[j] * (vabs / r3 + 3.0 * fabs(rv) / (r2 * r2)));",
                        "nsum_add(&SJ, m[j] * (vabs / r3 + fabs(rv) / (r2 * r2)));"),
    "scale_sj_power": ("nsum_add(&SJ, m[j] * (vabs / r3 + 3.0 * fabs(rv) / (r2 * r2)));",
                       "nsum_add(&SJ, m[j] * (vabs / r2 + 3.0 * fabs(rv) / (r2 * r2)));"),
    "scale_sj_signed_rv": ("nsum_add(&SJ, m[j] * (vabs / r3 + 3.0 * fabs(rv) / (r2 * r2)));",
                           "nsum_add(&SJ, m[j] * (vabs / r3 + 3.0 * rv / (r2 * r2)));"),
    "irr_scale_sa_power": ("nsum_add(&SA, mj / d2);", "nsum_add(&SA, mj / d3);"),
    "irr_scale_sj_factor": ("nsum_add(&SJ, mj * (vabs / d3 + 3.0 * fabs(rdotv) / (d2 * d2)));",
                            "nsum_add(&SJ, mj * (vabs / d3 + fabs(rdotv) / (d2 * d2)));"),
    # regular corrector
    "corr_no_list_correction": ("const double dF = (f_new[k] - f_old[k]) + (g_new[k] - g_old[k]);",
                                "const double dF = (f_new[k] - f_old[k]);"),
    "corr_list_correction_sign": ("const double dF = (f_new[k] - f_old[k]) + (g_new[k] - g_old[k]);",
                                  "const double dF = (f_new[k] - f_old[k]) - (g_new[k] - g_old[k]);"),
    "corr_f3_factor": ("F3[c] = (-12.0 * dF + 6.0 * h * (2.0 * fd_old[k] + dFd)) / (h * h * h);",
                       "F3[c] = (-12.0 * dF + 6.0 * h * (1.0 * fd_old[k] + dFd)) / (h * h * h);"),
    "corr_f2_at_old_time": ("F2[c] = f2_old + h * F3[c];", "F2[c] = f2_old;"),
    "corr_no_doubling_limit": ("const double lim = fmin(fmin(est, 2.0 * h), dt_max);",
                               "const double lim = fmin(est, dt_max);"),
    "corr_not_commensurate": ("while (d > dt_min && (d > limit || fmod(t, d) != 0.0)) d *= 0.5;",
                              "while (d > dt_min && d > limit) d *= 0.5;"),
    "corr_eta_squared": ("sqrt(eta * (a * a2 + ad * ad)", "sqrt(eta * eta * (a * a2 + ad * ad)"),
    "corr_radius_inverse": ("cbrt(n_p[q] / (double)nnb[q])", "cbrt((double)nnb[q] / n_p[q])"),
    "corr_radius_no_limit": ("f = fmin(fmax(cbrt(n_p[q] / (double)nnb[q]), f_lo), f_hi);",
                             "f = cbrt(n_p[q] / (double)nnb[q]);"),
    # potential
    "pot_sign": ("nsum_add(&PHI, -m[j] / r);", "nsum_add(&PHI, m[j] / r);"),
    "pot_inverse_square": ("nsum_add(&PHI, -m[j] / r);", "nsum_add(&PHI, -m[j] / r2);"),
    "pot_mass_of_i": ("nsum_add(&PHI, -m[j] / r);", "nsum_add(&PHI, -m[i] / r);"),
    "pot_includes_neighbours": ("++count;\n                continue;",
                                "++count;\n                nsum_add(&PHI, -m[j] / sqrt(r2));\n                continue;"),
    "irr_pot_sign": ("nsum_add(&PHI, -mj / d);", "nsum_add(&PHI, mj / d);"),
    "irr_pot_power": ("nsum_add(&PHI, -mj / d);", "nsum_add(&PHI, -mj / d2);"),
    # irregular force
    "irr_R_sign": ("Rij[c] = xp[3 * j + c] - xp[3 * i + c];", "Rij[c] = xp[3 * i + c] - xp[3 * j + c];"),
    "irr_V_sign": ("Vij[c] = vp[3 * j + c] - vp[3 * i + c];", "Vij[c] = vp[3 * i + c] - vp[3 * j + c];"),
    "irr_mass_of_i": ("const double mj = m[j];", "const double mj = m[i];"),
    "irr_drop_rv_term": ("mj * (Vij[c] / d3 - 3.0 * rdotv * Rij[c] / d5)", "mj * (Vij[c] / d3)"),
    "irr_jerk_rv_sign": ("mj * (Vij[c] / d3 - 3.0 * rdotv * Rij[c] / d5)",
                         "mj * (Vij[c] / d3 + 3.0 * rdotv * Rij[c] / d5)"),
    "irr_d3_as_d2": ("double d3 = d2 * d;", "double d3 = d2;"),
    "irr_d5_as_d4": ("double d5 = d3 * d2;", "double d5 = d2 * d2;"),
    "irr_skip_first_entry": ("for (int64_t e = 0; e < cnt[q]; ++e) {\n            const int64_t j",
                             "for (int64_t e = 1; e < cnt[q]; ++e) {\n            const int64_t j"),
    "irr_last_entry_dropped": ("for (int64_t e = 0; e < cnt[q]; ++e) {\n            const int64_t j",
                               "for (int64_t e = 0; e + 1 < cnt[q]; ++e) {\n            const int64_t j"),
    "irr_self_not_skipped": ("const int64_t j = list[q * lcap + e];\n            if (j == i) continue;",
                             "const int64_t j = list[q * lcap + e];"),
    "irr_wrong_row": ("const int64_t j = list[q * lcap + e];", "const int64_t j = list[e];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    path = tmp_path / "mut.c"
    path.write_text(mutated)
    so = str(tmp_path / f"libmut_{name}.so")
    oracle.build(str(path), so)
    lib = oracle.oracle._load(so)
    failed = None
    for pin in P.ALL_PINS:  # cheapest first; the first failure settles it
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts
            failed = (pin.__name__, type(e).__name__)
            break
    assert failed, f"mutant {name} passed every pin"
