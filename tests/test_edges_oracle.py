"""Pins of the oracle's threshold edges (graph slices of Section 5).

The weights the paper prints for its worked example, the plain definition
(brute-force alignment scores and exact fractions) on tiny dictionaries, and
the histogram of the top-k oracle fix the edge sets; planted mistakes in the
slice test must fail one of them.  CPU only.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle
from conftest import read_golden
from oracle import brute


def _puisant():
    g = {}
    for k, v in read_golden("puisant.txt"):
        g.setdefault(k, []).append(v)
    names = ["puisant", "paysans", "epuisant"]
    words = [[int(x) for x in g[k][0]] for k in names]
    syms = np.array([s for w in words for s in w], np.uint8)
    offs = np.cumsum([0] + [len(w) for w in words]).astype(np.uint64)
    sim = oracle.sim_matrix(int(g["alphabet"][0][0]), int(g["match"][0][0]), int(g["mismatch"][0][0]))
    return names, words, syms, offs, sim, int(g["gap"][0][0]), g


def _edge_set(i, j, s):
    return {(int(a), int(b), int(c)) for a, b, c in zip(i, j, s)}


def test_paper_normalised_weights_and_slices():
    names, words, syms, offs, sim, gap, g = _puisant()
    ix = {k: t for t, k in enumerate(names)}
    # the weights printed in Section 5: 300/5 = 60 and 200/3 (about 66.7)
    w_pp = oracle.normalised_weight(oracle.score(words[0], words[1], sim, gap), len(words[0]), len(words[1]))
    w_pe = oracle.normalised_weight(oracle.score(words[0], words[2], sim, gap), len(words[0]), len(words[2]))
    assert w_pp == 60 and w_pe == Fraction(200, 3)
    for a, b, num, den in g["normalised"]:
        assert oracle.normalised_weight(oracle.score(words[ix[a]], words[ix[b]], sim, gap),
                                        len(words[ix[a]]), len(words[ix[b]])) == Fraction(int(num), int(den))
    # slices through those weights select exactly the stated edges
    e = _edge_set(*oracle.edges(syms, offs, sim, gap, 60, 60, normalised=True))
    assert e == {(0, 1, 3)}
    e = _edge_set(*oracle.edges(syms, offs, sim, gap, 200, 200, normalised=True, den=3))
    assert e == {(0, 2, 4)}
    e = _edge_set(*oracle.edges(syms, offs, sim, gap, 60, 100, normalised=True))
    assert {(0, 1, 3), (0, 2, 4)} <= e
    # 66 < 200/3 < 67: the edge to epuisant is in [66, 67] but not in [67, 100] or [60, 66]
    assert (0, 2, 4) in _edge_set(*oracle.edges(syms, offs, sim, gap, 66, 67, normalised=True))
    assert (0, 2, 4) not in _edge_set(*oracle.edges(syms, offs, sim, gap, 67, 100, normalised=True))
    assert (0, 2, 4) not in _edge_set(*oracle.edges(syms, offs, sim, gap, 60, 66, normalised=True))
    # raw slices on the printed scores 3 and 4
    assert _edge_set(*oracle.edges(syms, offs, sim, gap, 4, 4)) == {(0, 2, 4)}
    assert {(0, 1, 3), (0, 2, 4)} <= _edge_set(*oracle.edges(syms, offs, sim, gap, 3, 4))


def _tiny_dict(rng, n, lmax, alphabet, allow_empty=True):
    lens = rng.integers(0 if allow_empty else 1, lmax + 1, size=n)
    words = [list(rng.integers(0, alphabet, size=L)) for L in lens]
    syms = np.array([s for w in words for s in w], np.uint8)
    offs = np.cumsum([0] + [len(w) for w in words]).astype(np.uint64)
    return words, syms, offs


SLICES = [
    (False, -3, 1, 1), (False, 0, 0, 1), (False, -100, 100, 1),
    (True, 0, 100, 1), (True, -100, -34, 1), (True, 40, 49, 1), (True, 200, 200, 3), (True, -101, 33, 2),
]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_edges_match_the_plain_definition(seed):
    """Brute-force alignment scores and exact fractions on tiny dictionaries."""
    rng = np.random.default_rng(100 + seed)
    words, syms, offs = _tiny_dict(rng, 9, 5, 3)
    gap = [-1, -2, -1][seed]
    sim = oracle.sim_matrix(3, 1, -1) if seed < 2 else np.array([[2, -1, 0], [-1, 1, -3], [0, -3, 3]], np.int32)
    n = len(words)
    truth = {}
    for a, b in itertools.combinations(range(n), 2):
        truth[(a, b)] = brute.brute_score(words[a], words[b], sim, gap)
    for normalised, lo, hi, den in SLICES:
        want = set()
        for (a, b), s in truth.items():
            if normalised:
                w = Fraction(100 * s, max(len(words[a]), len(words[b]), 1))
                ok = Fraction(lo, den) <= w <= Fraction(hi, den)
            else:
                ok = lo <= s <= hi
            if ok:
                want.add((a, b, s))
        got = _edge_set(*oracle.edges(syms, offs, sim, gap, lo, hi, normalised, den))
        assert got == want, (normalised, lo, hi, den)
        # an index range keeps exactly the edges whose row-major pair index falls in it
        E = n * (n - 1) // 2
        b0, b1 = E // 3, 2 * E // 3
        part = _edge_set(*oracle.edges(syms, offs, sim, gap, lo, hi, normalised, den, b0, b1))
        assert part == {(a, b, s) for (a, b, s) in want if b0 <= a * (2 * n - a - 1) // 2 + (b - a - 1) < b1}


def test_raw_slices_partition_and_agree_with_the_histogram():
    rng = np.random.default_rng(7)
    words, syms, offs = _tiny_dict(rng, 60, 7, 5, allow_empty=False)
    sim = oracle.sim_matrix(5, 1, -1)
    n = len(words)
    lo, hi = oracle.score_bounds(7, sim, -1)
    _, _, hist = oracle.topk_rows(syms, offs, sim, -1, 4, hist_range=(lo, hi))
    total = 0
    for s in range(lo, hi + 1):
        i, j, sc = oracle.edges(syms, offs, sim, -1, s, s)
        assert len(i) == int(hist[s - lo])
        assert np.all(sc == s) and np.all(i < j)
        total += len(i)
    assert total == n * (n - 1) // 2


_REAL_IN_SLICE = oracle.in_slice

MUTANTS = {
    # normalised by the shorter word
    "min_length": lambda s, la, lb, lo, hi, normalised=False, den=1: _REAL_IN_SLICE(
        s, np.minimum(la, lb), np.minimum(la, lb), lo, hi, normalised, den),
    # the factor 100 dropped
    "no_percent": lambda s, la, lb, lo, hi, normalised=False, den=1: (
        _REAL_IN_SLICE(s, la, lb, lo, hi, False, den) if not normalised else
        (np.asarray(s) * den >= lo * np.maximum(np.maximum(la, lb), 1)) &
        (np.asarray(s) * den <= hi * np.maximum(np.maximum(la, lb), 1))),
    # the upper end of the slice left open
    "open_upper_end": lambda s, la, lb, lo, hi, normalised=False, den=1: _REAL_IN_SLICE(
        s, la, lb, lo, hi, normalised, den) & ~_REAL_IN_SLICE(s, la, lb, hi, hi, normalised, den),
    # the denominator applied to the wrong side
    "den_inverted": lambda s, la, lb, lo, hi, normalised=False, den=1: _REAL_IN_SLICE(
        s, la, lb, lo * den * den, hi * den * den, normalised, den) if normalised else _REAL_IN_SLICE(
        s, la, lb, lo, hi, normalised, den),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_slice_mutants(name, monkeypatch):
    monkeypatch.setattr(oracle, "in_slice", MUTANTS[name])
    caught = []
    for t in (test_paper_normalised_weights_and_slices,
              lambda: [test_edges_match_the_plain_definition(s) for s in range(3)],
              test_raw_slices_partition_and_agree_with_the_histogram):
        try:
            t()
        except AssertionError:
            caught.append(t)
    assert caught, f"no pin caught mutant {name}"
