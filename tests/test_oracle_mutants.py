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
    "first_column_not_gapped": ("M[i * W + 0] = gap * (int32_t)i;", "M[i * W + 0] = 0;"),
    "first_row_wrong_sign": ("M[0 * W + j] = gap * (int32_t)j;", "M[0 * W + j] = -gap * (int32_t)j;"),
    "diag_wrong_index": ("M[(i - 1) * W + (j - 1)] + cost", "M[(i - 1) * W + j] + cost"),
    "delete_drops_gap": ("M[(i - 1) * W + j] + gap;", "M[(i - 1) * W + j];"),
    "insert_wrong_neighbour": ("M[i * W + (j - 1)] + gap;", "M[(i - 1) * W + (j - 1)] + gap;"),
    "sim_transposed": ("sim[(int64_t)A[i - 1] * alphabet + B[j - 1]]",
                       "sim[(int64_t)B[j - 1] * alphabet + A[i - 1]]"),
    "symbol_off_by_one": ("sim[(int64_t)A[i - 1] * alphabet + B[j - 1]]",
                          "sim[(int64_t)A[i % la] * alphabet + B[j - 1]]"),
    "max_becomes_min": ("if (deleteScore > best) best = deleteScore;",
                        "if (deleteScore < best) best = deleteScore;"),
    "wrong_result_cell": ("return M[la * W + lb];", "return M[la * W + (lb > 0 ? lb - 1 : 0)];"),
    "tie_break_reversed": ("return a->index < b->index ? -1 : 1;", "return a->index > b->index ? -1 : 1;"),
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
