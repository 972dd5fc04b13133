"""The pins must catch plausible mistakes in the oracle.

Each mutant is a copy of oracle/nw_oracle.c with one planted mistake (a dropped
term, a wrong sign or index, a transposed operand, a reversed tie-break ...),
built into a temporary library.  The pin tests are then run against it with
the oracle's library handle swapped; at least one of them must fail.
Everything here runs on the CPU.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "nw_oracle.c")

MUTANTS = {
    "first_column_not_gapped": ("int32_t left = (int32_t)i * gap;", "int32_t left = 0;"),
    "first_row_wrong_sign": ("line[j] = (int32_t)j * gap;", "line[j] = -(int32_t)j * gap;"),
    "diag_uses_left_cell": ("int32_t v = corner + sim", "int32_t v = left + sim"),
    "left_not_advanced": ("            left = v;\n", ""),
    "corner_not_advanced": ("            corner = above;\n", ""),
    "a_gap_drops_penalty": ("const int32_t a_gapped = above + gap;", "const int32_t a_gapped = above;"),
    "b_gap_wrong_neighbour": ("const int32_t b_gapped = left + gap;", "const int32_t b_gapped = corner + gap;"),
    "sim_transposed": ("sim[(int64_t)A[i - 1] * alphabet + B[j - 1]]",
                       "sim[(int64_t)B[j - 1] * alphabet + A[i - 1]]"),
    "symbol_off_by_one": ("sim[(int64_t)A[i - 1] * alphabet + B[j - 1]]",
                          "sim[(int64_t)A[i % la] * alphabet + B[j - 1]]"),
    "max_becomes_min": ("if (a_gapped > v) v = a_gapped;", "if (a_gapped < v) v = a_gapped;"),
    "wrong_result_cell": ("return line[lb];", "return line[lb > 0 ? lb - 1 : 0];"),
    "tie_break_reversed": ("return j < e->index;", "return j > e->index;"),
    "full_list_keeps_every_offer": ("if (k == 0 || !comes_before(s, j, &list[k - 1])) return;",
                                    "if (k == 0) return;"),
    "insertion_skips_shift": ("while (p > 0 && comes_before(s, j, &list[p - 1])) {",
                              "while (p > 1 && comes_before(s, j, &list[p - 1])) {"),
    "self_loop_kept": ("if (J->kind == JOB_TOPK && j == i) continue;", ""),
    "hist_counts_both_directions": ("J->kind == JOB_TOPK && j > i)", "J->kind == JOB_TOPK && j != i)"),
    "triangle_row_start_wrong": ("- (uint64_t)(r - 1) * (uint64_t)r / 2u;", "- (uint64_t)r * (uint64_t)r / 2u;"),
}

PIN_TESTS = [
    pins.test_puissance_nuance_worked_example,
    pins.test_puisant_pairs_section5,
    pins.test_oracle_equals_brute_force_random_up_to_6,
    pins.test_asymmetric_matrix_orientation,
    pins.test_self_score_symmetry_empty_and_bounds,
    pins.test_textbook_special_cases,
    pins.test_triangle_pairs_topk_query_agree_with_single_scores,
    pins.test_duplicate_words_are_distinct_neighbours,
]


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC, encoding="utf-8").read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path_c = tmp_path / f"{name}.c"
    path_c.write_text(src.replace(old, new), encoding="utf-8")
    path_so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-w",
                           "-o", str(path_so), str(path_c)])
    return str(path_so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    so = _build_mutant(tmp_path, name, old, new)
    saved = oracle._load()
    try:
        oracle._lib = None
        lib = ctypes.CDLL(so)
        # reuse the argument declarations of the real library
        for fn in ("orc_score1", "orc_matrix", "orc_triangle", "orc_pairs", "orc_topk_rows", "orc_query"):
            getattr(lib, fn).restype = getattr(saved, fn).restype
            getattr(lib, fn).argtypes = getattr(saved, fn).argtypes
        oracle._lib = lib
        caught = []
        for t in PIN_TESTS:
            try:
                t()
            except AssertionError:
                caught.append(t.__name__)
        assert caught, f"no pin caught mutant {name}"
    finally:
        oracle._lib = saved
