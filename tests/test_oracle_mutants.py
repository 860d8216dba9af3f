"""The pins of test_oracle_pins.py must reject a plausible mistake in each
reading they pin.  Each case copies the oracle's C source, plants one mistake
by a textual edit, builds the copy with the oracle's flags, and runs the pin
that must catch it against that copy (the real oracle is untouched).
"""
import math
import os

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_rungs as rungs
import test_oracle_sources as sources


def _mutant(tmp_path, name, edits):
    src = oracle.source()
    for old, new in edits:
        assert src.count(old) >= 1, (name, old)
        src = src.replace(old, new)
    return oracle.build_variant(src, str(tmp_path / f"liborc_{name}.so"))


SWAP_PSI = [("qL[q] = orc_pair_limit(qL[q], qi[q], qj[q], p->psi1, p->psi2);",
             "qL[q] = orc_pair_limit(qL[q], qi[q], qj[q], p->psi2, p->psi1);"),
            ("qR[q] = orc_pair_limit(qR[q], qj[q], qi[q], p->psi1, p->psi2);",
             "qR[q] = orc_pair_limit(qR[q], qj[q], qi[q], p->psi2, p->psi1);")]
SWAP_PSI_INSIDE = [("double d1 = psi1 * dq, d2 = psi2 * dq;",
                    "double d1 = psi2 * dq, d2 = psi1 * dq;")]
NO_PREDICTOR = [("0.5 * dt, 0.5 * dt, c,", "0.0 * dt, 0.0 * dt, c,")]
START_FRAME = [("double vf[3] = {0.5 * (qpi[Q_VX] + qpj[Q_VX]), 0.5 * (qpi[Q_VY] + qpj[Q_VY]),",
                "double vf[3] = {0.5 * (qi[Q_VX] + qj[Q_VX]), 0.5 * (qi[Q_VY] + qj[Q_VY]),"),
               ("0.5 * (qpi[Q_VZ] + qpj[Q_VZ])};", "0.5 * (qi[Q_VZ] + qj[Q_VZ])};")]
WRONG_UPWIND = [("const double *wu = (us >= 0.0) ? wL : wR;",
                 "const double *wu = (us >= 0.0) ? wR : wL;")]
BETA_INVERTED = [("double t = (p->ncond_max - nc) / (p->ncond_max - 1.0);",
                  "double t = (nc - 1.0) / (p->ncond_max - 1.0);")]
NO_HALF = [("double ex = 0.5 * (g[q][0] * d[0]", "double ex = 1.0 * (g[q][0] * d[0]")]


def test_swapped_psi_at_the_face_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "swap_psi", SWAP_PSI)):
        with pytest.raises(AssertionError):
            pins.test_face_uses_the_pair_limited_states()


def test_swapped_psi_in_the_limiter_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "swap_psi_inside", SWAP_PSI_INSIDE)):
        with pytest.raises(AssertionError):
            pins.test_pair_limiter_branches(*pins.PAIR_CASES[0])


def test_wrong_upwind_side_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "upwind", WRONG_UPWIND)):
        with pytest.raises(AssertionError):
            pins.test_mfv_face_flux_is_the_moving_surface_flux(*pins.FACE_STATES[0])


def test_inverted_beta_ramp_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "beta", BETA_INVERTED)):
        with pytest.raises(AssertionError):
            pins.test_conditioned_bj_limiter_by_hand(0.14, (20.0, 80.0))


def test_full_step_extrapolation_in_the_limiter_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "nohalf", NO_HALF)):
        with pytest.raises(AssertionError):
            pins.test_conditioned_bj_limiter_by_hand(0.1, (1.0, 1.0))


def _order(scheme):
    e16, _ = pins.oracle_soundwave_L1(16, scheme)
    e32, _ = pins.oracle_soundwave_L1(32, scheme)
    return math.log2(e16 / e32)


@pytest.mark.parametrize("name,edits", [("no_predictor", NO_PREDICTOR),
                                        ("start_of_step_frame", START_FRAME)])
def test_first_order_time_integration_is_caught(tmp_path, name, edits):
    with oracle.use_library(_mutant(tmp_path, name, edits)):
        order = _order("mfv")
    print(name, f"MFV order {order:.2f}")
    assert order < 1.8


ETA_PRINTED = [("const double eta_u = 1.5 * (gam - 1.0);", "const double eta_u = 1.5;")]
GWORK_SIGN = [("gwork[(int64_t)k * n + a] += dm * d[k];", "gwork[(int64_t)k * n + a] -= dm * d[k];")]
# S~ taken after the gravity kick (momentum P~ + m a dt) instead of at the hydro update
KICKED_SOURCE = [("(p0[2] + p1[2]) * a3[2]);", "(p0[2] + p1[2] + dt * m1 * a3[2]) * a3[2]);")]


def test_hubble_eta_of_the_list_is_caught(tmp_path):
    # eta = 3/2 for U, as listed beside the equations: u ~ a^-3, not the adiabat a^-2
    with oracle.use_library(_mutant(tmp_path, "eta", ETA_PRINTED)):
        with pytest.raises(AssertionError):
            sources.test_comoving_adiabatic_expansion_second_order(1e30)


def test_mass_exchange_work_sign_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "gwork", GWORK_SIGN)):
        with pytest.raises(AssertionError):
            sources.test_mass_exchange_work_identity()


def test_source_at_the_kicked_state_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "kick", KICKED_SOURCE)):
        with pytest.raises(AssertionError):
            sources.test_free_fall_in_a_uniform_field()


# individual time steps (sec. 2.3.4, sec. 2.3.10)
FACE_DT_MAX = [("const int rf = rung[a] > rung[b] ? rung[a] : rung[b];",
                "const int rf = rung[a] < rung[b] ? rung[a] : rung[b];")]
NO_LIMITER = [("      if (*ra < *rb - 2) {", "      if (0) {"),
              ("      if (*rb < *ra - 2) {", "      if (0) {")]
RUNG_NOT_STRICT = [("    if (dti > s) return r;", "    if (dti >= s) return r;")]
NO_DRIFT = [("xn += (double)(k - s0[i]) * delta * v[i];", "xn += 0.0;")]


def test_face_step_of_the_larger_rung_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "facedt", FACE_DT_MAX)):
        with pytest.raises(AssertionError):
            rungs.test_mixed_rungs_track_global_steps()


def test_missing_rung_limiter_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "nolimiter", NO_LIMITER)):
        with pytest.raises(AssertionError):
            rungs.test_rung_limiter_is_the_least_fixed_point()


def test_non_strict_rung_criterion_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "strict", RUNG_NOT_STRICT)):
        with pytest.raises(AssertionError):
            rungs.test_rung_is_the_smallest_power_of_two()


def test_inactive_particles_left_behind_is_caught(tmp_path):
    with oracle.use_library(_mutant(tmp_path, "nodrift", NO_DRIFT)):
        with pytest.raises(AssertionError):
            rungs.test_moving_lattice_on_random_rungs_moves_rigidly("mfm")
