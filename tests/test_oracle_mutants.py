"""Plants plausible mistakes (a dropped term, a wrong sign or operand, an
off-by-one, a changed tie-break) in a private copy of the oracle's C source,
builds it, and checks that the pins of the other test files reject every
mutant.  Runs only on the CPU and never touches the GPU library."""
import os
import subprocess
import sys

import pytest

import oracle
import test_oracle_assign as ta
import test_oracle_ccl as tc
import test_oracle_lab as tl
import test_oracle_net as tn
import test_oracle_seed as ts
import test_oracle_update as tu
import test_oracle_variants as tv

SRC = os.path.join(os.path.dirname(oracle.__file__), "slic_oracle.c")
NET_SRC = os.path.join(os.path.dirname(oracle.__file__), "net_oracle.c")

# (name, original text, mutated text, pins expected to notice)
MUTANTS = [
    ("a_sign", "float dxy = fx - fy;", "float dxy = fy - fx;", ["lab"]),
    ("matrix_swap", "{0.4124, 0.3576, 0.1805}", "{0.4124, 0.1805, 0.3576}", ["lab"]),
    ("linear_segment", "r = s / 116.0;", "r = s / 161.0;", ["lab"]),
    ("cbrt_step", "double err = fma(-g, y3, 1.0);", "double err = fma(-g, y3, 1.001);", ["lab"]),
    ("gradient_dropped_term", "B[d] - B[u]", "B[d] - B[d]", ["seed"]),
    ("gradient_clamp", "xl = x > 0 ? x - 1 : 0", "xl = x > 0 ? x - 1 : 1", ["seed"]),
    ("seed_tiebreak", "if (g < gbest)", "if (g <= gbest)", ["seed"]),
    ("seed_middle", "sx = x0 + (x1 - x0 - 1) / 2", "sx = x0 + (x1 - x0) / 2", ["seed"]),
    ("distance_operand", "db = c[2] - b;\n    float dlab", "db = c[2] - a;\n    float dlab",
     ["assign"]),
    ("distance_weight", "float sp = wgt * dxy;", "float sp = dxy;", ["assign"]),
    ("distance_dy", "dy = c[4] - (float)y;\n    float s = dx * dx;",
     "dy = c[4] - (float)x;\n    float s = dx * dx;", ["assign"]),
    ("distance_sq_weight", "float w2 = wgt * wgt;", "float w2 = wgt;", ["variants"]),
    ("xyz_scale", "C1[i] = 100.0f * Y;", "C1[i] = 10.0f * Y;", ["variants"]),
    ("assign_tiebreak", "if (bk < 0 || d < best)", "if (bk < 0 || d <= best)", ["assign"]),
    ("assign_window", "for (int32_t dx = -1; dx <= 1; dx++) {\n                    int32_t cx",
     "for (int32_t dx = -1; dx <= 0; dx++) {\n                    int32_t cx", ["assign"]),
    ("update_y_sum", "s[4] += y;", "s[4] += x;", ["update"]),
    ("update_divisor", "double mean = (double)s[j] / n;", "double mean = (double)s[j] / (n + 1);",
     ["update"]),
    ("update_empty", "if (counts[k] == 0) continue;", "", ["update"]),
    ("update_rounding", "s[1] += llrintf(A[i] * scale);", "s[1] += (int64_t)(A[i] * scale);",
     ["update"]),
    ("loop_extra_round", "for (int32_t it = 0; it < iters; it++)",
     "for (int32_t it = 0; it <= iters; it++)", ["update"]),
    ("update_votes_ignored", "if (votes && !votes[i]) continue;", "", ["votes"]),
    ("ccl_join_direction", "size_t q = x > 0 ? r - 1 : r - (size_t)w;",
     "size_t q = x > 0 ? r - (size_t)w : r - 1;", ["ccl"]),
    ("ccl_threshold", "(int64_t)4 * size[r] < (int64_t)S * (int64_t)S",
     "(int64_t)4 * size[r] <= (int64_t)S * (int64_t)S", ["ccl"]),
    ("ccl_pixel0", "if (r != 0 && small)", "if (small)", ["ccl"]),
    ("energy_divisor", "*out = acc / ((double)w * (double)h);",
     "*out = acc / ((double)w * (double)h + 1.0);", ["ccl"]),
]

# mistakes planted in the warm-start net oracle
NET_MUTANTS = [
    ("net_tap_transposed", "                    int xx = x + t % 3 - 1, yy = y + t / 3 - 1;\n"
     "                    if (xx < 0 || yy < 0 || xx >= n->w",
     "                    int xx = x + t / 3 - 1, yy = y + t % 3 - 1;\n"
     "                    if (xx < 0 || yy < 0 || xx >= n->w", ["net"]),
    ("net_phase_axes", "int ph = ((y + n->oy) % n->S) * n->S + (x + n->ox) % n->S;",
     "int ph = ((x + n->ox) % n->S) * n->S + (y + n->oy) % n->S;", ["net"]),
    ("net_relu_mask", "if (!(n.a2[i] > 0.0)) d2[i] = 0.0;", "", ["net"]),
    ("net_softmax_grad", "d[c] = (pr - (c == target[i] ? 1.0 : 0.0))",
     "d[c] = (pr - (c == target[i] ? 0.5 : 0.0))", ["net"]),
    ("net_input_scale", "n->x[3 * i + 1] = rnd(bf, (double)(A[i] / 128.0f));",
     "n->x[3 * i + 1] = rnd(bf, (double)(A[i] / 100.0f));", ["net"]),
    ("votes_direction", "votes[i] = s * tau <= 1.0;", "votes[i] = s * tau >= 1.0;", ["net"]),
    ("votes_reference_class", "for (int c = 0; c < C3; c++) s += exp(l[c] - l[best]);",
     "for (int c = 0; c < C3; c++) s += exp(l[c] - l[0]);", ["net"]),
    ("votes_dropped_term", "for (int c = 0; c < C3; c++) s += exp(l[c] - l[best]);",
     "for (int c = 1; c < C3; c++) s += exp(l[c] - l[best]);", ["net"]),
]

PINS = {
    "lab": [tl.test_white_is_exactly_100_0_0, tl.test_black, tl.test_published_colorimetry,
            tl.test_neutral_axis],
    "seed": [lambda: ts.test_planted_minimum_is_found(),
             lambda: ts.test_gradient_definition_on_known_values(),
             lambda: [ts.test_seeds_sit_in_cell_middles_on_a_flat_image(37, 29, 8, p)
                      for p in (False, True)],
             lambda: [ts.test_seed_perturbation_bruteforce(s) for s in range(12)]],
    "assign": [lambda: [ta.test_assignment_bruteforce(s, m) for s in range(6)
                        for m in (0.0, 10.0, 40.0)],
               ta.test_exact_ties_go_to_lowest_index,
               lambda: [ta.test_uniform_image_gives_the_grid(12, 12, 3, i) for i in (0, 1)]],
    "update": [lambda: [tu.test_update_is_the_exact_mean(s) for s in range(6)],
               tu.test_zero_iterations_is_one_association_with_the_seeds,
               lambda: tu.test_uniform_image_centres_land_on_cell_middles(15, 9, 3)],
    "net": [lambda: [tn.test_backward_matches_central_differences(s) for s in range(2)],
            lambda: [tn.test_forward_matches_scipy_correlation(s) for s in range(2)],
            lambda: [tn.test_votes_closed_form(t) for t in (0.2, 0.5, 0.7, 0.9)],
            tn.test_votes_against_softmax],
    "votes": [lambda: [tu.test_update_over_voting_pixels_is_their_exact_mean(s)
                       for s in range(3)]],
    "variants": [tv.test_xyz_white_black_grey, tv.test_xyz_is_additive_over_the_primaries,
                 lambda: [tv.test_squared_association_is_the_nearest_candidate(m)
                          for m in (10.0, 40.0)],
                 tv.test_squared_energy_is_the_mean_root],
    "ccl": [lambda: [tc.test_matches_independent_statement(s) for s in range(40)],
            lambda: [tc.test_invariants(s) for s in range(5)],
            lambda: [tc.test_energy_is_the_mean_eq1_distance(s) for s in range(3)]],
}


def _caught(pins) -> bool:
    for fn in pins:
        try:
            fn()
        except (AssertionError, ValueError, IndexError):
            return True
    return False


_RUNNER = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle
oracle._LIB = {lib!r}
import test_oracle_mutants as tm
pins = [p for g in {groups!r} for p in tm.PINS[g]]
sys.exit(3 if tm._caught(pins) else 0)
"""


@pytest.mark.parametrize("name,orig,mut,groups", MUTANTS + NET_MUTANTS,
                         ids=[m[0] for m in MUTANTS + NET_MUTANTS])
def test_pins_reject_mutant(tmp_path, name, orig, mut, groups):
    """Each mutant runs in a child process, so one that crashes (an index
    gone out of range) counts as rejected without taking pytest down."""
    target = NET_SRC if groups == ["net"] else SRC
    src = open(target).read()
    assert src.count(orig) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(orig, mut))
    other = tmp_path / "other.c"
    other.write_text(open(SRC if target == NET_SRC else NET_SRC).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, str(path), str(other), "-o", str(lib), "-lm"],
                   check=True)
    tests = os.path.dirname(os.path.abspath(__file__))
    code = _RUNNER.format(root=os.path.dirname(tests), tests=tests, lib=str(lib), groups=groups)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300)
    assert res.returncode != 0, f"mutant {name} passed every pin"
    # 3: a pin failed; negative: the mutant crashed (killed by a signal)
    assert res.returncode == 3 or res.returncode < 0, res.stderr.decode()[-2000:]
