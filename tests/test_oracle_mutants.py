"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
the pins catch every one of them.  This is what makes the pins evidence: each
mutation below is a slip that could plausibly be made in the real oracle."""
import pytest

from oracle import oracle as O
import tests.test_oracle_pins as P

# (name, text in the oracle source, replacement, pins expected to catch it)
MUTANTS = [
    ("field_h_not_halved", "0.5 * (double)in->h[i]", "1.0 * (double)in->h[i]",
     [P.test_zero_couplings_closed_form]),
    ("update_sign_flipped", "double t = tanh(phi[i] / T);", "double t = -tanh(phi[i] / T);",
     [lambda: P.test_free_energy_is_nonincreasing_over_sweeps("lattice2d", 1.0),
      lambda: P.test_brute_force_ground_state_is_reached("sk16")]),
    ("dense_field_wrong_index", "s += (double)row[j] * x[j];", "s += (double)row[j] * x[i];",
     [lambda: P.test_gauge_covariance_bitwise("phased", 2)]),
    ("lattice_backward_bond_wrong_site", "w[n++] = (double)in->bond[(size_t)a * in->N + jm];",
     "w[n++] = (double)in->bond[(size_t)a * in->N + i];",
     [lambda: P.test_free_energy_is_nonincreasing_over_sweeps("lattice2d", 1.0)]),
    ("energy_drops_field", "acc_add(&a, -(double)in->h[i] * si);", "(void)si;",
     [P.test_energy_dense_real_couplings_exact]),
    ("rounding_ties_away", "if (round_bit && (sticky || (sig & 1)))", "if (round_bit)",
     [P.test_exact_sum_matches_fsum_and_fractions]),
    ("geometric_ratio_inverted", "log(sc->T_end / T0)", "log(T0 / sc->T_end)",
     [P.test_geometric_levels]),
    ("rng_constant", "0xBF58476D1CE4E5B9ull", "0xBF58476D1CE4E5B8ull",
     [P.test_splitmix64_published_vector]),
    ("convergence_test_inverted", ": (!(d < sc->d_min) && sweeps < sc->max_sweeps));",
     ": ((d < sc->d_min) && sweeps < sc->max_sweeps));",
     [P.test_fixed_point_residual_after_convergence]),
    ("linear_schedule_relaxes_at_T0", "double t = T0;", "double t = T0 + sc->c_step;",
     [P.test_linear_levels_paper_schedule]),
    ("csr_field_wrong_column", "s += (double)in->val[k] * x[in->col[k]];", "s += (double)in->val[k] * x[k % in->N];",
     [lambda: P.test_free_energy_is_nonincreasing_over_sweeps("er", 1.0)]),
    ("checkerboard_wrong_parity", "phase_of[i] = sum & 1;", "phase_of[i] = (i & 1);",
     [P.test_phase_partitions]),
    ("damping_weights_swapped", "(1.0 - g) * m[i] + g * t;", "g * m[i] + (1.0 - g) * t;",
     [lambda: P.test_zero_couplings_damped_closed_form(0.3)]),
    ("cap_counted_at_one_sweep", "if (sc->max_sweeps > 1 && !(d < sc->d_min))", "if (!(d < sc->d_min))",
     [P.test_cap_hits_count_levels_cut_by_the_cap]),
    ("cap_never_counted", "++cap; /* a level cut short by the sweep cap */", "/* cap dropped */",
     [P.test_cap_hits_count_levels_cut_by_the_cap]),
    ("stop_one_sweep_late", "if (!own && ((d < sc->d_min) || sweeps >= sc->max_sweeps)) {",
     "if (!own && sweeps > 1 && ((d < sc->d_min) || sweeps >= sc->max_sweeps)) {",
     [P.test_replay_of_own_counts_and_of_other_counts]),
    ("best_ties_highest_index", "if (best < 0 || energy[r] < energy[best])",
     "if (best < 0 || energy[r] <= energy[best])", [P.test_best_run_ties_lowest_index]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    src = O.source()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    path = O.build_variant(src.replace(old, new), str(tmp_path / ("lib_" + name + ".so")))
    caught = False
    with O.use_library(path):
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught = True
    assert caught, name + " was not caught"
