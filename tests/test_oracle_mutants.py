"""The pins must catch plausible mistakes in the oracle.

Each case compiles a copy of the oracle's C source with one planted mistake (a
dropped term, a wrong sign, index, coefficient or condition) into a temporary
directory, points the oracle module at that copy, and runs the pin that should
fail.  Everything here runs on the CPU; the real oracle is restored afterwards.
"""
import os
import subprocess

import pytest

import oracle as real_oracle
import test_oracle_blocksteps as tb
import test_oracle_energy as te
import test_oracle_force as tf
import test_oracle_hermite as th
import test_oracle_hermite6 as t6
import test_oracle_groups as tg
import test_fp32_floor as tfl

SRC = os.path.join(os.path.dirname(real_oracle.__file__), "nbody_oracle.c")

MUTANTS = [
    ("jerk drops the radial term", "cs_add(&jk[d], mu * (w[d] - alpha * r[d]))", "cs_add(&jk[d], mu * (w[d]))",
     lambda o: tf.test_jerk_is_time_derivative_of_acc(o, 3)),
    ("jerk coefficient 2 instead of 3", "3.0 * rw * rinv2", "2.0 * rw * rinv2",
     lambda o: tf.test_jerk_is_time_derivative_of_acc(o, 3)),
    ("pair vector reversed", " r[d] = x[3 * j + d] - x[3 * i + d];", " r[d] = x[3 * i + d] - x[3 * j + d];",
     lambda o: tf.test_acc_is_minus_gradient_of_potential(o, 0)),
    ("mass of i instead of j", "m[j] * rinv * rinv2", "m[i] * rinv * rinv2",
     lambda o: tf.test_acc_is_minus_gradient_of_potential(o, 0)),
    ("eps instead of eps^2", "r[2] * r[2] + eps2;", "r[2] * r[2] + eps;",
     lambda o: tf.test_acc_is_minus_gradient_of_potential(o, 0)),
    ("kinetic energy missing the half", "cs_add(&kin, 0.5 * m[i] * v2)", "cs_add(&kin, m[i] * v2)",
     lambda o: te.test_circular_binary_virial_and_kepler_energy(o, 0.5, 0.5, 1.0)),
    ("potential halved", "cs_add(&p, m[i] * m[j] / sqrt(r2 + eps2))", "cs_add(&p, 0.5 * m[i] * m[j] / sqrt(r2 + eps2))",
     lambda o: te.test_potential_gradient_matches_force(o)),
    ("potential ignores softening", "sqrt(r2 + eps2))", "sqrt(r2))",
     lambda o: te.test_potential_gradient_matches_force(o)),
    ("predictor a d^2/6", "a[q] * d * d / 2.0", "a[q] * d * d / 6.0",
     lambda o: th.test_predictor_is_exact_for_cubic_motion(o)),
    ("predictor drops jerk in v", "vp[q] = v[q] + a[q] * d + jk[q] * d * d / 2.0;", "vp[q] = v[q] + a[q] * d;",
     lambda o: th.test_predictor_is_exact_for_cubic_motion(o)),
    ("corrector jerk weights swapped", "h * (4.0 * j0 + 2.0 * j1)", "h * (2.0 * j0 + 4.0 * j1)",
     lambda o: th.test_corrector_is_exact_for_quintic_motion(o, 2.0 ** -4)),
    ("corrector a3 h^5/24", "h * h * h * h * h / 120.0", "h * h * h * h * h / 24.0",
     lambda o: th.test_corrector_is_exact_for_quintic_motion(o, 0.5)),
    ("corrector sign of a3 term", "a3[c] = (12.0 * (a0 - a1) + 6.0 * h * (j0 + j1))",
     "a3[c] = (12.0 * (a0 - a1) - 6.0 * h * (j0 + j1))",
     lambda o: th.test_kepler_orbit_matches_closed_form(o, 0.5, 1e-5)),
    ("Aarseth numerator |j| instead of |j|^2", "an * sn + jn * jn", "an * sn + jn",
     lambda o: th.test_aarseth_step_on_circular_orbit(o)),
    ("Aarseth without sqrt", "dta = sqrt(eta * num / den);", "dta = eta * num / den;",
     lambda o: th.test_aarseth_step_on_circular_orbit(o)),
    ("doubling ignores commensurability", "fmod(t_next, 2.0 * h) == 0.0", "1",
     lambda o: tb.test_block_step_invariants_over_a_run(o)),
    ("select takes everything due within twice the block time", "if (t[i] + dt[i] == tn)", "if (t[i] + dt[i] <= 2.0 * tn)",
     lambda o: tb.test_select_against_brute_scan(o)),
    ("startup step not a power of two", "        dt[i] = step;\n    }\n    return 0;", "        dt[i] = want;\n    }\n    return 0;",
     lambda o: th.test_aarseth_step_on_circular_orbit(o)),
    # 6th-order scheme
    ("snap drops the 3 beta A term", "- 3.0 * beta * Ad", "",
     lambda o: t6.test_snap_is_second_time_derivative_of_acc(o, 5)),
    ("snap coefficient 3 instead of 6", "6.0 * alpha * Jd", "3.0 * alpha * Jd",
     lambda o: t6.test_snap_is_second_time_derivative_of_acc(o, 5)),
    ("snap uses relative velocity for relative acceleration", "mu * aij[d]", "mu * vij[d]",
     lambda o: t6.test_snap_is_second_time_derivative_of_acc(o, 5)),
    ("beta without alpha^2", "+ alpha * alpha;", ";",
     lambda o: t6.test_snap_is_second_time_derivative_of_acc(o, 5)),
    ("predictor crackle c d^5/24", "cr[q] * tau * tau * tau * tau * tau / 120.0",
     "cr[q] * tau * tau * tau * tau * tau / 24.0",
     lambda o: t6.test_predictor6_is_exact_for_quintic_motion(o)),
    ("predicted acceleration drops snap", "ap[q] = a[q] + jk[q] * tau + sn[q] * tau * tau / 2.0",
     "ap[q] = a[q] + jk[q] * tau",
     lambda o: t6.test_predictor6_is_exact_for_quintic_motion(o)),
    ("corrector6 snap weight h^3/60", "h * h * h / 120.0 * (s0 + s1)", "h * h * h / 60.0 * (s0 + s1)",
     lambda o: t6.test_corrector6_is_exact_for_quartic_acceleration(o, 0.5)),
    ("corrector6 jerk difference reversed", "- h * h / 10.0 * (j1 - j0)", "- h * h / 10.0 * (j0 - j1)",
     lambda o: t6.test_corrector6_is_exact_for_quartic_acceleration(o, 2.0 ** -4)),
    ("corrector6 position uses a jerk difference", "h * h * h / 120.0 * (j0 + j1)",
     "h * h * h / 120.0 * (j1 - j0)",
     lambda o: t6.test_corrector6_is_exact_for_quartic_acceleration(o, 0.5)),
    ("interpolant condition row", "{3.0, 4.0, 5.0}", "{3.0, 4.0, 6.0}",
     lambda o: t6.test_corrector6_velocity_and_crackle_exact_for_quintic_acceleration(o, 0.5)),
    ("crackle coefficient 30 instead of 60", "60.0 * k5 * h * h", "30.0 * k5 * h * h",
     lambda o: t6.test_corrector6_velocity_and_crackle_exact_for_quintic_acceleration(o, 0.5)),
    ("criterion ratio under a square root", "double dta = den_c > 0.0 ? eta * (num / den_c) : INFINITY;",
     "double dta = den_c > 0.0 ? eta * sqrt(num / den_c) : INFINITY;",
     lambda o: t6.test_generalized_step_on_circular_orbits(o, 0.5)),
    ("criterion denominator without |s|", "const double den_c = sN + sqrt(jn * cn);",
     "const double den_c = 0.0 + sqrt(jn * cn);",
     lambda o: t6.test_generalized_step_on_circular_orbits(o, 2.0)),
    ("criterion numerator without |j|", "const double num = sqrt(an * sN) + jn;",
     "const double num = sqrt(an * sN);",
     lambda o: t6.test_generalized_step_on_circular_orbits(o, 2.0)),
    ("criterion without the crackle", "const double den_c = sN + sqrt(jn * cn);",
     "const double den_c = den_d;",
     lambda o: t6.test_close_encounter_in_a_strong_field_is_resolved(o, 0.1, 1e-6)),
    ("criterion without the floor", "        if (dta < dtd / 8.0)\n            dta = dtd / 8.0;", "",
     lambda o: t6.test_force_noise_does_not_shrink_a_small_shared_step(o)),
    ("6th-order startup ignores the snap",
     "        double want = (bottom > 0.0) ? eta_s * (top / bottom) : dt_max;",
     "        double want = (jn > 0.0) ? eta_s * an / jn : dt_max;",
     lambda o: t6.test_close_encounter_in_a_strong_field_is_resolved(o, 0.01, 5e-9)),
    ("6th-order startup |j|/|a| instead of |j|^2/|a|",
     "const double bottom = sm + (an > 0.0 ? jn * jn / an : 0.0);",
     "const double bottom = sm + (an > 0.0 ? jn / an : 0.0);",
     lambda o: t6.test_generalized_step_on_circular_orbits(o, 2.0)),
    # tight groups
    ("tidal tensor without the isotropic term", "- (a == b ? 1.0 : 0.0) / s32", "",
     lambda o: tg.test_tidal_is_minus_hessian_of_potential(o, 7)),
    ("tidal tensor factor 2 instead of 3", "m[j] * (3.0 * d[a] * d[b] / s52", "m[j] * (2.0 * d[a] * d[b] / s52",
     lambda o: tg.test_tidal_is_minus_hessian_of_potential(o, 7)),
    ("Kepler drift g without the time", "const double g = (Mrem - (x - sx)) / nmean;",
     "const double g = (0.0 - (x - sx)) / nmean;",
     lambda o: tg.test_kepler_drift_matches_closed_form(o, 0.3, 1.7)),
    ("Kepler drift sign of sigma term", "+ se * (1.0 - cos(x)) - Mrem;", "- se * (1.0 - cos(x)) - Mrem;",
     lambda o: tg.test_kepler_drift_matches_closed_form(o, 0.3, 1.7)),
    ("Kepler solver without its bracket", "        if (!(xn > lo && xn < hi))\n            xn = 0.5 * (lo + hi);\n", "",
     lambda o: tg.test_kepler_drift_invariants_at_high_eccentricity(o)),
    ("tidal kick of the wrong sign", "v[a] += 0.5 * h * tr;", "v[a] -= 0.5 * h * tr;",
     lambda o: tg.test_group_advance_conserves_the_jacobi_integral_of_a_constant_tide(o)),
    ("tidal kicks at the substep start only", "const double w = half == 0 ? wa : wb;", "const double w = wa;",
     lambda o: tg.test_group_advance_is_second_order(o)),
    ("nearest keeps the last of equal distances", "                if (d < bd) {", "                if (d <= bd) {",
     lambda o: tg.test_nearest_is_the_brute_force_scan(o)),
    ("nearest counts the body itself", "            if (j == i)\n                    continue;\n                const double dx", "            if (0)\n                    continue;\n                const double dx",
     lambda o: tg.test_nearest_is_the_brute_force_scan(o)),
    ("tidal at points leaves out only the first body", "if (j == excl[2 * k] || j == excl[2 * k + 1])", "if (j == excl[2 * k])",
     lambda o: tg.test_tidal_at_points_is_minus_hessian_of_the_rest(o)),
    ("tidal at points measured from the origin", "d[c] = x[3 * j + c] - p[3 * k + c];", "d[c] = x[3 * j + c];",
     lambda o: tg.test_tidal_at_points_is_minus_hessian_of_the_rest(o)),
    ("velocity scale without |v_j|", "cs_add(&t, m[j] * (vi + vj) / (s * sqrt(s)));",
     "cs_add(&t, m[j] * vi / (s * sqrt(s)));",
     lambda o: tfl.test_velocity_scale_is_the_plain_sum(o)),
    ("velocity scale with s^-1 instead of s^-3/2", "cs_add(&t, m[j] * (vi + vj) / (s * sqrt(s)));",
     "cs_add(&t, m[j] * (vi + vj) / s);",
     lambda o: tfl.test_velocity_scale_is_the_plain_sum(o)),
    ("velocity scale counts the body itself",
     "            if (j == i)\n                continue;\n            double dr[3];",
     "            if (0)\n                continue;\n            double dr[3];",
     lambda o: tfl.test_velocity_scale_is_the_plain_sum(o)),
]


def _load(path):
    """Bind a mutant library with the same signatures as the real one."""
    saved_lib, saved_path = real_oracle._lib, real_oracle._LIB_PATH
    real_oracle._lib, real_oracle._LIB_PATH = None, path
    orig_build = real_oracle.build
    real_oracle.build = lambda force=False: path
    try:
        return real_oracle.lib()
    finally:
        real_oracle.build = orig_build
        real_oracle._lib, real_oracle._LIB_PATH = saved_lib, saved_path


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must match exactly once: %r" % old
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", so, str(mutant), "-lm"], check=True)
    mlib = _load(so)
    real_oracle.build(force=False)
    saved = real_oracle._lib
    real_oracle._lib = mlib
    try:
        with pytest.raises((AssertionError, real_oracle.OracleError)):
            pin(real_oracle)
    finally:
        real_oracle._lib = saved


def test_unmutated_oracle_passes_the_same_pins():
    real_oracle.build(force=False)
    for _, _, _, pin in MUTANTS:
        pin(real_oracle)
