"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's C source, builds it,
and runs, in a fresh interpreter against that build, the pins named for it:
every one of them must fail (the same pins without the planted mistake run
in the rest of the suite). The mistakes: a dropped or doubled factor in the
push, a wrong divisor, a threshold without the degree, a different log base,
a wrong constant, a missing case of eqn:rmax, a wrong walk weight, an
inverted stop test, a biased neighbour choice, walks keyed without their
index, a weight credited to the start instead of the end point, a broken
Philox key schedule and a reversed tie order in the top-k."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fora_oracle.c")
P = "tests/test_oracle_pins.py::"
GOLDEN = P + "test_push_golden_synchronous_rounds"
INVARIANT = P + "test_push_invariant_uniform"

# mistake: (text in the oracle's source, text planted instead, pins that catch it)
MUTATIONS = {
    "reserve_without_alpha": ("q[v] += alpha * x[i];", "q[v] += x[i];", [GOLDEN, INVARIANT]),
    "increment_damped_twice": (
        "double inc = ((1.0 - alpha) * x[i]) / (double)d;",
        "double inc = ((1.0 - alpha) * (1.0 - alpha) * x[i]) / (double)d;", [GOLDEN, INVARIANT]),
    "increment_over_d_plus_one": (
        "double inc = ((1.0 - alpha) * x[i]) / (double)d;",
        "double inc = ((1.0 - alpha) * x[i]) / (double)(d + 1);", [GOLDEN, INVARIANT]),
    "threshold_without_degree": (
        "double thr = rmax * (double)(rowptr[v + 1] - rowptr[v]);", "double thr = rmax;",
        [GOLDEN, P + "test_push_invariant_rmat"]),
    "log_base_2": ("double L = log(2.0 / pf);", "double L = log2(2.0 / pf);",
                   [P + "test_omega_meets_lemma2_bound"]),
    "wrong_c": ("double c = 2.0 * eps / 3.0 + 2.0;", "double c = 2.0 * eps / 3.0 + 1.0;",
                [P + "test_omega_meets_lemma2_bound"]),
    "rmax_without_case_2": (
        "if ((double)m * rmax > 1.0) rmax = (eps * eps) * delta / (c * L);", "",
        [P + "test_rmax_case_two"]),
    "weight_over_omega_unit": ("pw[e] = r[v] / om;", "pw[e] = r[v] / omega_unit;",
                               [P + "test_walk_totals"]),
    "stop_test_inverted": ("y[0] < t_alpha) break;", "y[0] >= t_alpha) break;",
                           [P + "test_walk_length_is_geometric"]),
    "neighbour_biased": ("x = colidx[rowptr[x] + (int64_t)idx];",
                         "x = colidx[rowptr[x] + (int64_t)(idx / 2)];",
                         [P + "test_walk_neighbour_choice_is_uniform"]),
    "walk_index_not_keyed": ("uint32_t ctr[4] = {(uint32_t)v, (uint32_t)j, b, 0u};",
                             "uint32_t ctr[4] = {(uint32_t)v, 0u, b, 0u};",
                             [P + "test_walk_length_is_geometric"]),
    "weight_at_start_node": ("acc[x] += pw[e];", "acc[v] += pw[e];",
                             [P + "test_walk_weight_lands_at_the_end_point"]),
    "philox_key_schedule": ("k1 += PHILOX_WEYL_1;", "k1 += PHILOX_WEYL_0;",
                            ["tests/test_philox_library.py::test_extreme_blocks"]),
    "topk_ties_descending": ("return (i > j) - (i < j);", "return (i < j) - (i > j);",
                             [P + "test_topk_matches_sort"]),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_a_planted_mistake(tmp_path, name):
    old, new, pins = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"the mutation site of {name} is not unique"
    src = tmp_path / "fora_oracle.c"
    src.write_text(text.replace(old, new))
    lib = tmp_path / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", "-o", str(lib), str(src), "-lm"],
                   check=True, capture_output=True, timeout=120)
    code = ("import sys; sys.path.insert(0, %r); import oracle; "
            "oracle._SRC = %r; oracle._LIB_PATH = %r; import pytest; "
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', *%r]))"
            % (ROOT, str(src), str(lib), pins))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                         text=True, timeout=300)
    # exit status 1: the pins ran and failed (not a usage or collection
    # error), and none of them passed
    assert out.returncode == 1, f"{name}: pins did not fail\n{out.stdout[-2000:]}"
    last = out.stdout.strip().splitlines()[-1]
    assert "failed" in last and "passed" not in last, last
