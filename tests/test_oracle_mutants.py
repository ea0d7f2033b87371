"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch each of them (CPU only; the planted copies live in a temporary folder)."""
import os

import pytest

import oracle
from oracle import build as obuild
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "dicod_oracle.c")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("eq3_sign_flipped",
     "s->beta[(int64_t)k * s->L + t] -= Srow[t - t0 + W - 1] * delta;",
     "s->beta[(int64_t)k * s->L + t] += Srow[t - t0 + W - 1] * delta;"),
    ("eq3_lag_reversed",
     "Srow[t - t0 + W - 1] * delta",
     "Srow[t0 - t + W - 1] * delta"),
    ("s_operands_transposed",
     "const double *Srow = s->S + IDX3(k, k0, 0, K, nd);",
     "const double *Srow = s->S + IDX3(k0, k, 0, K, nd);"),
    ("beta_updated_at_k0_t0",
     "if (k == k0 && t == t0)\n                continue;",
     "if (0)\n                continue;"),
    ("window_too_short",
     "int64_t hi = t0 + (W - 1) > s->L - 1 ? s->L - 1 : t0 + (W - 1);",
     "int64_t hi = t0 + (W - 2) > s->L - 1 ? s->L - 1 : t0 + (W - 2);"),
    ("no_norm_division",
     "double zp = oracle_soft_threshold(s->beta[i], s->lam) / s->n2[k];",
     "double zp = oracle_soft_threshold(s->beta[i], s->lam);"),
    ("no_norm_division_in_stop_test",
     "double zp = oracle_soft_threshold(beta[(int64_t)k * L + t], lam) / n2[k];",
     "double zp = oracle_soft_threshold(beta[(int64_t)k * L + t], lam);"),
    ("threshold_dropped",
     "double a = fabs(u) - lam;",
     "double a = fabs(u);"),
    ("convolution_instead_of_correlation",
     "s += D[IDX3(k, p, tau, P, W)] * Y[(int64_t)p * T + t + tau];",
     "s += D[IDX3(k, p, W - 1 - tau, P, W)] * Y[(int64_t)p * T + t + tau];"),
    ("norm_missing_in_beta",
     "beta[(int64_t)k * L + t] += n2[k] * Z[(int64_t)k * L + t];",
     "beta[(int64_t)k * L + t] += Z[(int64_t)k * L + t];"),
    ("neighbour_never_notified",
     "touch_r = 1;",
     "touch_r = 0;"),
    ("prop_a1_beta_term_sign",
     "b0 * (z_old - z_new) + s->lam",
     "-b0 * (z_old - z_new) + s->lam"),
    ("objective_half_dropped",
     "return 0.5 * quad + lam * l1;",
     "return quad + lam * l1;"),
    ("interference_lag_reversed",
     "st->interf_sum += s->S[IDX3(u->k0, v->k0, dt + W - 1, K, nd)] *",
     "st->interf_sum += s->S[IDX3(u->k0, v->k0, -dt + W - 1, K, nd)] *"),
    ("h1_includes_zero_shift",
     "if (d == 0)\n                    continue;\n                double r",
     "if (0)\n                    continue;\n                double r"),
    ("h1_unnormalised",
     "/ sqrt(n2[k] * n2[l]);",
     "/ 1.0;"),
    ("gap_safe_theta_not_rescaled",
     "const double sc = cmax > lam ? cmax : lam;",
     "const double sc = lam;"),
    ("gap_safe_radius_halved",
     "const double r = sqrt(2.0 * G) / lam;",
     "const double r = sqrt(0.5 * G) / lam;"),
    ("gap_safe_atom_norm_dropped",
     "fabs(c[i]) / sc + r * sqrt(n2[k]) < 1.0",
     "fabs(c[i]) / sc + r < 1.0"),
    ("message_sent_to_wrong_side",
     "out[((size_t)(m + 1) * 2) * per + n_out[2 * (m + 1)]++] = msg;",
     "out[((size_t)(m + 1) * 2 + 1) * per + n_out[2 * (m + 1)]++] = msg;"),
]


def _pins():
    rows = pins._read_golden()
    return [
        lambda: pins.test_soft_threshold_hand_values(),
        lambda: pins.test_s_table_matches_numpy_correlate(),
        lambda: pins.test_correlate_matches_numpy(),
        lambda: pins.test_reconstruct_matches_numpy_convolve(),
        lambda: pins.test_beta_matches_definition_with_replacement_operator(),
        lambda: pins.test_single_segment_is_greedy_cd(0),
        lambda: pins.test_prop_a1_cost_change_matches_objective(),
        lambda: pins.test_monotone_decrease_and_lemma_a1_bound(),
        lambda: pins.test_orthonormal_atoms_of_length_one_closed_form(),
        lambda: pins.test_single_coordinate_closed_form(),
        lambda: [pins.test_golden_two_coordinate_lasso(r) for r in rows],
        lambda: pins.test_tiny_brute_force_explicit_toeplitz_lasso(0),
        lambda: pins.test_kkt_conditions_at_solution(),
        lambda: pins.test_scaled_atoms_explicit_toeplitz_lasso(0),
        lambda: pins.test_max_dz_matches_definition_scaled_atoms(),
        lambda: pins.test_dicod_schedule_cost_identity(1, 4, 3),
        lambda: pins.test_dicod_schedule_interferes_and_converges(),
        lambda: pins.test_h1_ratio_closed_forms(),
        lambda: pins.test_h1_ratio_matches_numpy_definition(),
        lambda: pins.test_gap_safe_closed_form_at_zero(),
        lambda: pins.test_gap_safe_is_safe_and_bounds_the_objective(0),
        lambda: pins.test_gap_safe_mask_is_the_sphere_test(),
    ]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    msrc = tmp_path / "mutant.c"
    msrc.write_text(mutated)
    lib = obuild.build(src=str(msrc), lib=str(tmp_path / "libmutant.so"))
    prev = oracle.use_library(oracle.load_library(lib))
    real_lgcd = oracle.lgcd

    def bounded_lgcd(*a, **kw):        # a broken solver may never stop
        kw["max_steps"] = min(kw.get("max_steps", 10**9), 20000)
        return real_lgcd(*a, **kw)

    oracle.lgcd = bounded_lgcd
    caught = []
    try:
        for i, pin in enumerate(_pins()):
            try:
                pin()
            except AssertionError:
                caught.append(i)
            except Exception:           # a crash of the mutant counts as caught
                caught.append(i)
    finally:
        oracle.lgcd = real_lgcd
        oracle.use_library(prev)
    assert caught, f"no pin caught the planted mistake '{name}'"
