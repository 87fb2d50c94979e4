"""The oracle's pins catch plausible mistakes (CPU only).

Each case copies the oracle package, plants one mistake in one of its files
(the C core, the Python driver of the next rows, or the MLP reference),
builds the copy, and runs, in a fresh interpreter that imports the copy, the
pins named for that mistake: every one of them must fail (the same pins
without the planted mistake run in the rest of the suite).

The mistakes cover the push (dropped, doubled or misplaced factors, a
threshold without the degree), the constants (log base, c, the second case
of eqn:rmax), the walks (weight, stop test, neighbour choice, keying, where
the weight lands, the Philox key schedule), the top-k tie order, Algorithm 3
(residue scaling, the alpha r start, the forced first move), Algorithm 5
(eps / 2, the split of p_f, the stopping test, the delta sequence), the
FORA+ index size, source distributions (estimate, walk key), the frontier
replay (its push test, final check; its rounds share the push's code) and the MLP
reference (GELU derivative, loss gradient, Adam's bias correction, BF16
ties, a feature)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
P = "tests/test_oracle_pins.py::"
A3 = "tests/test_alg3_oracle.py::"
TK = "tests/test_topk_oracle.py::"
LO = "tests/test_learned_oracle.py::"
GOLDEN = P + "test_push_golden_synchronous_rounds"
INVARIANT = P + "test_push_invariant_uniform"
C, PY, MLP = "fora_oracle.c", "__init__.py", "mlp.py"

# mistake: (file, text in it, text planted instead, pins that catch it)
MUTATIONS = {
    "reserve_without_alpha": (C, "q[v] += alpha * x[i];", "q[v] += x[i];", [GOLDEN, INVARIANT]),
    "increment_damped_twice": (
        C, "double inc = ((1.0 - alpha) * x[i]) / (double)d;",
        "double inc = ((1.0 - alpha) * (1.0 - alpha) * x[i]) / (double)d;", [GOLDEN, INVARIANT]),
    "increment_over_d_plus_one": (
        C, "double inc = ((1.0 - alpha) * x[i]) / (double)d;",
        "double inc = ((1.0 - alpha) * x[i]) / (double)(d + 1);", [GOLDEN, INVARIANT]),
    "threshold_without_degree": (
        C, "double thr = rmax * (double)(rowptr[v + 1] - rowptr[v]);", "double thr = rmax;",
        [GOLDEN, P + "test_push_invariant_rmat"]),
    "log_base_2": (C, "double L = log(2.0 / pf);", "double L = log2(2.0 / pf);",
                   [P + "test_omega_meets_lemma2_bound"]),
    "wrong_c": (C, "double c = 2.0 * eps / 3.0 + 2.0;", "double c = 2.0 * eps / 3.0 + 1.0;",
                [P + "test_omega_meets_lemma2_bound"]),
    "rmax_without_case_2": (
        C, "if ((double)m * rmax > 1.0) rmax = (eps * eps) * delta / (c * L);", "",
        [P + "test_rmax_case_two"]),
    "weight_over_omega_unit": (C, "pw[e] = r[v] / om;", "pw[e] = r[v] / omega_unit;",
                               [P + "test_walk_totals"]),
    "stop_test_inverted": (C, "y[0] < t_alpha) break;", "y[0] >= t_alpha) break;",
                           [P + "test_walk_length_is_geometric"]),
    "neighbour_biased": (C, "x = colidx[rowptr[x] + (int64_t)idx];",
                         "x = colidx[rowptr[x] + (int64_t)(idx / 2)];",
                         [P + "test_walk_neighbour_choice_is_uniform"]),
    "walk_index_not_keyed": (C, "uint32_t ctr[4] = {(uint32_t)v, (uint32_t)j, b, 0u};",
                             "uint32_t ctr[4] = {(uint32_t)v, 0u, b, 0u};",
                             [P + "test_walk_length_is_geometric"]),
    "weight_at_start_node": (C, "acc[x] += pw[e];", "acc[v] += pw[e];",
                             [P + "test_walk_weight_lands_at_the_end_point"]),
    "philox_key_schedule": (C, "k1 += PHILOX_WEYL_1;", "k1 += PHILOX_WEYL_0;",
                            ["tests/test_philox_library.py::test_extreme_blocks"]),
    "topk_ties_descending": (C, "return (i > j) - (i < j);", "return (i < j) - (i > j);",
                             [P + "test_topk_matches_sort"]),
    "alg3_walk_residue_unscaled": (
        PY, 'r_walk = (1.0 - alpha) * ps["r"] if prune else ps["r"]', 'r_walk = ps["r"]',
        [A3 + "test_pruned_monte_carlo_case"]),
    "alg3_start_without_alpha_r": (
        PY, 'pi = ps["q"] + wk["acc"] + (alpha * ps["r"] if prune else 0.0)',
        'pi = ps["q"] + wk["acc"]', [A3 + "test_pruned_monte_carlo_case"]),
    "alg3_no_forced_move": (
        PY, 'wk = walks(g, k0, k1, c["t_alpha"], pv, po, pw, first_move=prune)',
        'wk = walks(g, k0, k1, c["t_alpha"], pv, po, pw, first_move=False)',
        [A3 + "test_pruned_query_walks_move_at_least_once"]),
    "topk_full_eps": (PY, "out = fora(g, s, alpha=alpha, eps=eps / 2,",
                      "out = fora(g, s, alpha=alpha, eps=eps,",
                      [TK + "test_iterations_hold_the_union_bound"]),
    "topk_pf_not_split": (PY, "pf_it = pf / (n * max(math.log2(n / k), 1.0))", "pf_it = pf",
                          [TK + "test_iterations_hold_the_union_bound"]),
    "topk_stop_without_eps": (
        PY, "if kth >= (1 + eps) * d or i == len(deltas) - 1:",
        "if kth >= d or i == len(deltas) - 1:", [TK + "test_definition_2_and_stopping_threshold"]),
    "topk_delta_quartered": (PY, "        d /= 2.0", "        d /= 4.0",
                             [TK + "test_delta_sequence"]),
    "index_floor": (PY, "om = np.ceil(deg * walks_per_degree).astype(np.uint64)",
                    "om = np.floor(deg * walks_per_degree).astype(np.uint64)",
                    ["tests/test_index_oracle.py::test_index_size_and_contents"]),
    "dist_estimate_without_reserve": (
        PY, '    pi = q + wk["acc"]\n', '    pi = wk["acc"]\n',
        ["tests/test_dist_oracle.py::test_point_mass_is_the_single_source_query"]),
    "dist_walk_key": (
        PY, 'wk = walks(g, DIST_KEY0, seed, c["t_alpha"], pv, po, pw)',
        'wk = walks(g, 0, seed, c["t_alpha"], pv, po, pw)',
        ["tests/test_dist_oracle.py::test_point_mass_is_the_single_source_query"]),
    "replay_listed_test_inverted": (
        C, "double rel = listed[v] ? (thr - r[v]) / thr : (r[v] - thr) / thr;",
        "double rel = listed[v] ? (r[v] - thr) / thr : (thr - r[v]) / thr;",
        ["tests/test_replay_oracle.py::test_replay_of_own_frontiers_is_bit_exact"]),
    "replay_without_final_check": (
        C, "double rel = (r[v] - thr) / thr;\n      if (rel > excess) excess = rel;", "",
        ["tests/test_replay_oracle.py::test_wrong_frontiers_are_reported"]),
    "mlp_gelu_grad_term": (MLP, "return _cdf(z) + z * _phi(z)", "return _cdf(z)",
                           [LO + "test_gelu_closed_forms",
                            LO + "test_backward_matches_finite_differences"]),
    "mlp_loss_gradient_halved": (
        MLP, "d3 = 2.0 * (y - np.asarray(t, np.float64)) / N",
        "d3 = (y - np.asarray(t, np.float64)) / N",
        [LO + "test_backward_matches_finite_differences"]),
    "mlp_adam_no_bias_correction": (MLP, "mh = m[sl] / (1 - b1 ** step)", "mh = m[sl]",
                                    [LO + "test_adam_first_step_moves_by_lr"]),
    "mlp_bf16_no_ties_to_even": (MLP, "r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16",
                                 "r = (u + 0x7FFF) >> 16", [LO + "test_bf16_rounding_cases"]),
    "mlp_feature_max_degree": (MLP, "math.log(dn.sum())", "math.log(dn.max())",
                               [LO + "test_features_hand_worked"]),
}


def _run_pins_on_copy(tmp_path, pins, mutation=None):
    """Copy the oracle package (planting `mutation` = (file, old, new) if
    given), build the copy and run `pins` against it in a fresh interpreter."""
    pkg = tmp_path / "oracle"
    shutil.copytree(ORACLE, pkg, ignore=shutil.ignore_patterns("__pycache__", "*.so*"))
    if mutation is not None:
        fname, old, new = mutation
        target = pkg / fname
        text = target.read_text()
        assert text.count(old) == 1, "the mutation site is not unique"
        target.write_text(text.replace(old, new))
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", "-o", str(pkg / "liboracle.so"), str(pkg / C), "-lm"],
                   check=True, capture_output=True, timeout=120)
    code = ("import sys; sys.path.insert(0, %r); import oracle; "
            "assert oracle.__file__.startswith(%r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', *%r]))"
            % (str(tmp_path), str(pkg), ROOT, pins))
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                          text=True, timeout=300)


@pytest.mark.slow
def test_the_unmodified_copy_passes_every_named_pin(tmp_path):
    pins = sorted({p for m in MUTATIONS.values() for p in m[3]})
    out = _run_pins_on_copy(tmp_path, pins)
    assert out.returncode == 0, out.stdout[-2000:]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_a_planted_mistake(tmp_path, name):
    fname, old, new, pins = MUTATIONS[name]
    out = _run_pins_on_copy(tmp_path, pins, (fname, old, new))
    # exit status 1: the pins ran and failed (not a usage or collection
    # error), and none of them passed
    assert out.returncode == 1, f"{name}: pins did not fail\n{out.stdout[-2000:]}"
    last = out.stdout.strip().splitlines()[-1]
    assert "failed" in last and "passed" not in last, last
