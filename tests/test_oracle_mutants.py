"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of hs_oracle.c (source substitution,
built with gcc into a temporary library, on the CPU), swaps it in, and checks
that at least one pin of tests/test_oracle_pins.py fails.  The real oracle is
restored afterwards.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "hs_oracle.c")

MUTANTS = {
    # floor replaced by C truncation on negative template indices
    "truncating_division": ("    if (q * b > a) q -= 1;\n", "\n"),
    # wrong row centre for even plane heights
    "row_centre": ("    int64_t c = T / 2;\n    return fdiv(r - c, m) + c;",
                   "    int64_t c = (T - 1) / 2;\n    return fdiv(r - c, m) + c;"),
    # the stretch plane SP_k dropped from the fp32 recursion
    "dropped_term": ("cur[r * N + j] = (k == 1) ? sp : prev[r * N + j] + sp;",
                     "cur[r * N + j] = (k == 1) ? sp : prev[r * N + j] + (k == 2 ? 0.0f : sp);"),
    # the bin of the stretch factor taken from the previous plane's factor
    "wrong_bin_index": ("float sp = fop[rs * ld + fdiv(j, k)];          /* SP_k(i,j) */",
                        "float sp = fop[rs * ld + fdiv(j, k > 2 ? k - 1 : k)];"),
    # rows and bins stretched the other way round (row not divided)
    "rows_not_stretched": ("int64_t rs = src_row(r, k, T);\n            for (int64_t j = 0; j < N; j++) {\n                float sp = fop[rs * ld + fdiv(j, k)];          /* SP_k(i,j) */",
                           "int64_t rs = r;\n            for (int64_t j = 0; j < N; j++) {\n                float sp = fop[rs * ld + fdiv(j, k)];          /* SP_k(i,j) */"),
    # non-strict threshold test in the detector
    "non_strict_threshold": ("n += (v > thr);", "n += (v >= thr);"),
    # plane field stores k instead of k-1
    "plane_field": ("hi = (uint32_t)(((uint64_t)r << (s_k + s_bin)) | ((uint64_t)(k - 1) << s_bin));",
                    "hi = (uint32_t)(((uint64_t)r << (s_k + s_bin)) | ((uint64_t)(k & 7) << s_bin));"),
    # detector reads the threshold of the wrong plane
    "threshold_plane": ("float thr = ta[(int64_t)(k - 1) * T + r] * scale;\n            int64_t n = 0;",
                        "float thr = ta[(int64_t)(k > 1 ? k - 2 : 0) * T + r] * scale;\n            int64_t n = 0;"),
    # transpose misses the largest stretch factor
    "vjp_dropped_term": ("for (int m = 1; m <= k; m++)\n                    dfop",
                         "for (int m = 1; m < k; m++)\n                    dfop"),
    # fractional variant: the point itself (m = k) left out
    "frac_last_term": ("    for (int m = 1; m <= k; m++) {\n        float x = fop[frac_row",
                       "    for (int m = 1; m < k; m++) {\n        float x = fop[frac_row"),
    # fractional variant: floor(i/k) * m instead of floor(m i/k) for rows
    "frac_row_product": ("    return fdiv(m * (r - c), k) + c;", "    return fdiv(r - c, k) * m + c;"),
    # fractional variant: m * floor(j/k) instead of floor(m j/k) for bins
    "frac_bin_product": ("float x = fop[frac_row(r, m, k, T) * ld + fdiv((int64_t)m * j, k)];",
                         "float x = fop[frac_row(r, m, k, T) * ld + (int64_t)m * fdiv(j, k)];"),
    # fractional variant: rows not stretched
    "frac_rows_unstretched": ("    return fdiv(m * (r - c), k) + c;", "    return r + 0 * m * k * c;"),
    # fractional variant: detection compares the wrong plane's threshold
    "frac_threshold_plane": ("        float thr = ta[(int64_t)(k - 1) * T + r] * scale;\n        int64_t n = 0;\n        for (int64_t j = 0; j < N; j++) n += (frac_point_f32",
                             "        float thr = ta[(int64_t)(k > 1 ? k - 2 : 0) * T + r] * scale;\n        int64_t n = 0;\n        for (int64_t j = 0; j < N; j++) n += (frac_point_f32"),
    # fp64 planes summed with a wrong sign
    "f64_sign": ("double sp = fop[rs * ld + fdiv(j, k)];\n                cur[r * N + j] = (k == 1) ? sp : prev[r * N + j] + sp;",
                 "double sp = fop[rs * ld + fdiv(j, k)];\n                cur[r * N + j] = (k == 1) ? sp : prev[r * N + j] - sp;"),
}


def _pin_calls():
    T64 = lambda: oracle.touch_counts(64, 1 << 12, 8, [8])  # noqa: E731
    return [
        lambda: pins.test_integer_planes_exact(21, 1024),
        lambda: pins.test_integer_planes_exact(64, 300),
        lambda: pins.test_random_planes_within_summation_bound(9, 333, 16),
        pins.test_point_definition,
        pins.test_example_point_sources,
        lambda: pins.test_algorithm2_order_bitwise(5, 64, 8),
        pins.test_k1_identity_and_detection,
        pins.test_monotone_in_k,
        lambda: pins.test_injected_harmonic_sums(-1),
        lambda: pins.test_touch_max_204(T64()),
        lambda: pins.test_touch_zoom_share(T64()),
        lambda: pins.test_touch_equals_transpose_with_unit_cotangent(T64()),
        pins.test_detect_matches_thresholded_planes,
        pins.test_tiny_workload_detects_all_injected_fundamentals,
        pins.test_packing_paper_formula,
        pins.test_vjp_scatter_equals_boxsum,
        pins.test_vjp_adjoint_identity,
        lambda: pins.test_frac_integer_planes_exact(9, 257, 16),
        pins.test_frac_k1_identity_and_k2_equals_paper,
        pins.test_frac_hand_points,
        lambda: pins.test_frac_harmonic_sum_closed_form(-1),
        pins.test_frac_detect_matches_thresholded_planes,
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "libm.so")
        open(c, "w").write(mutated)
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", so, c, "-lm"])
        saved = oracle._load()
        oracle._lib = oracle.load_library(so)
        failed = []
        try:
            for call in _pin_calls():
                try:
                    call()
                except (AssertionError, ValueError):
                    failed.append(call)
        finally:
            oracle._lib = saved
    assert failed, "no pin caught mutant " + name
