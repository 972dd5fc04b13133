"""Pins for the CPU oracle: paper values, brute force, invariants, special cases.

None of these compare the oracle with itself: each checks it against a value
the paper prints, a plain definition (every alignment enumerated), a textbook
routine written independently (edit distance, LCS) or an invariant the
mathematics fixes.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute
from conftest import read_golden

from synth import zipf_vocab, random_submat, uniform_vocab


def _golden_dict(rows):
    d = {}
    for k, v in rows:
        d.setdefault(k, []).append(v)
    return d


def _parse_alignment(tokens):
    cols = []
    for t in tokens:
        x, y = t.split(":")
        cols.append((brute.GAP if x == "-" else int(x), brute.GAP if y == "-" else int(y)))
    return cols


# ---------------------------------------------------------------- paper values

def test_puissance_nuance_worked_example():
    g = _golden_dict(read_golden("puissance_nuance.txt"))
    A = [int(x) for x in g["A"][0]]
    B = [int(x) for x in g["B"][0]]
    match, mismatch, gap = int(g["match"][0][0]), int(g["mismatch"][0][0]), int(g["gap"][0][0])
    sim = oracle.sim_matrix(40, match, mismatch)
    M = oracle.matrix(A, B, sim, gap)
    assert M.shape == (len(A) + 1, len(B) + 1)
    assert oracle.score(A, B, sim, gap) == int(g["score"][0][0])
    for i, j, v in g["cell"]:
        assert M[int(i), int(j)] == int(v), (i, j)
    # the first row and column are p times the index
    assert list(M[:, 0]) == [gap * i for i in range(len(A) + 1)]
    assert list(M[0, :]) == [gap * j for j in range(len(B) + 1)]
    # the two printed alignments score what the tables say
    opt = _parse_alignment(g["optimal_alignment"][0])
    other = _parse_alignment(g["other_alignment"][0])
    assert brute.alignment_score(opt, sim, gap) == int(g["optimal_alignment_score"][0][0])
    assert brute.alignment_score(other, sim, gap) == int(g["other_alignment_score"][0][0])
    # both are alignments of A and B, and brute force finds -2 as the maximum
    for cols in (opt, other):
        assert [x for x, _ in cols if x is not brute.GAP] == A
        assert [y for _, y in cols if y is not brute.GAP] == B
    assert brute.brute_score(A, B, sim, gap) == int(g["score"][0][0])
    enumerated = set(brute.alignments(A, B))
    assert tuple(other) in enumerated and tuple(opt) in enumerated
    assert len(enumerated) == brute.count_alignments(len(A), len(B))


def test_puisant_pairs_section5():
    g = _golden_dict(read_golden("puisant.txt"))
    words = {k: [int(x) for x in g[k][0]] for k in ("puisant", "paysans", "epuisant")}
    match, mismatch, gap = int(g["match"][0][0]), int(g["mismatch"][0][0]), int(g["gap"][0][0])
    sim = oracle.sim_matrix(int(g["alphabet"][0][0]), match, mismatch)
    for a, b, s in g["pair"]:
        assert oracle.score(words[a], words[b], sim, gap) == int(s)
        assert oracle.score(words[b], words[a], sim, gap) == int(s)
        assert brute.brute_score(words[a], words[b], sim, gap) == int(s)
    for a, b, num, den in g["normalised"]:
        s = oracle.score(words[a], words[b], sim, gap)
        assert 100 * s == int(num)
        assert max(len(words[a]), len(words[b])) == int(den)


# ---------------------------------------------------------------- brute force

SCORINGS = [
    ("pm1_gap1", dict(match=1, mismatch=-1), -1),
    ("pm1_gap2", dict(match=1, mismatch=-1), -2),
    ("lev", dict(match=0, mismatch=-1), -1),
    ("lcs", dict(match=1, mismatch=0), 0),
    ("cheap_gap", dict(match=2, mismatch=-5), -1),
]


@pytest.mark.parametrize("name,kw,gap", SCORINGS)
def test_oracle_equals_brute_force_all_short_words(name, kw, gap):
    """Every pair of words of length <= 3 over a 3-symbol alphabet."""
    sim = oracle.sim_matrix(3, **kw)
    words = [w for L in range(0, 4) for w in itertools.product(range(3), repeat=L)]
    for A in words:
        for B in words:
            assert oracle.score(A, B, sim, gap) == brute.brute_score(A, B, sim, gap), (A, B)


def test_oracle_equals_brute_force_random_up_to_6():
    rng = np.random.default_rng(11)
    sub = random_submat(6, seed=12)                      # symmetric, [-3,3], diag +3
    asym = rng.integers(-3, 4, size=(6, 6)).astype(np.int32)   # an asymmetric matrix too
    cases = [(oracle.sim_matrix(6, 1, -1), -1), (oracle.sim_matrix(6, submat=sub), -2),
             (oracle.sim_matrix(6, submat=asym), -1)]
    for sim, gap in cases:
        for _ in range(25):
            la, lb = rng.integers(0, 7, size=2)
            A = rng.integers(0, 6, size=la)
            B = rng.integers(0, 6, size=lb)
            assert oracle.score(A, B, sim, gap) == brute.brute_score(A, B, sim, gap)
    # the longest case: D(6,6) alignments
    A = [0, 1, 2, 3, 4, 5]
    B = [5, 1, 2, 0, 4, 3]
    assert brute.count_alignments(6, 6) == 8989
    assert sum(1 for _ in brute.alignments(A, B)) == 8989
    for sim, gap in cases:
        assert oracle.score(A, B, sim, gap) == brute.brute_score(A, B, sim, gap)


def test_asymmetric_matrix_orientation():
    """A indexes rows: sim[x][y] with x from A.  With an asymmetric matrix,
    swapping A and B must follow the transposed matrix."""
    sim = np.array([[0, 5], [-5, 0]], dtype=np.int32)
    assert oracle.score([0], [1], sim, -10) == 5
    assert oracle.score([1], [0], sim, -10) == -5
    assert oracle.score([1], [0], np.ascontiguousarray(sim.T), -10) == 5


# ---------------------------------------------------------------- invariants

def _random_words(rng, count, alphabet, maxlen):
    return [rng.integers(0, alphabet, size=rng.integers(0, maxlen + 1)) for _ in range(count)]


def test_self_score_symmetry_empty_and_bounds():
    rng = np.random.default_rng(5)
    sub = random_submat(64, seed=4)
    for sim, gap, match in [(oracle.sim_matrix(40, 1, -1), -1, 1), (oracle.sim_matrix(64, submat=sub), -2, 3)]:
        alphabet = sim.shape[0]
        words = _random_words(rng, 60, alphabet, 20)
        for A in words:
            assert oracle.score(A, A, sim, gap) == len(A) * match       # self score
            assert oracle.score(A, [], sim, gap) == len(A) * gap         # against the empty word
            assert oracle.score([], A, sim, gap) == len(A) * gap
        lo, hi = oracle.score_bounds(20, sim, gap)
        for A, B in zip(words[::2], words[1::2]):
            s = oracle.score(A, B, sim, gap)
            assert s == oracle.score(B, A, sim, gap)                     # symmetric S
            assert lo <= s <= hi


def test_pm1_identity_and_tight_bounds():
    """+1/-1/-1: 2 s = la + lb - min(4 mismatches + 3 gaps); -max <= s <= 2 min - max."""
    rng = np.random.default_rng(6)
    sim = oracle.sim_matrix(4, 1, -1)
    for _ in range(200):
        A = rng.integers(0, 4, size=rng.integers(0, 6))
        B = rng.integers(0, 4, size=rng.integers(0, 6))
        s = oracle.score(A, B, sim, -1)
        D = min(sum(4 if (x is not brute.GAP and y is not brute.GAP and x != y) else
                    (3 if (x is brute.GAP or y is brute.GAP) else 0) for x, y in cols)
                for cols in brute.alignments(A, B))
        assert 2 * s == len(A) + len(B) - D
        la, lb = len(A), len(B)
        assert -max(la, lb) <= s <= 2 * min(la, lb) - max(la, lb)


def test_textbook_special_cases():
    rng = np.random.default_rng(7)
    lev = oracle.sim_matrix(10, 0, -1)
    lcs = oracle.sim_matrix(10, 1, 0)
    for _ in range(300):
        A = rng.integers(0, 10, size=rng.integers(0, 21))
        B = rng.integers(0, 10, size=rng.integers(0, 21))
        assert oracle.score(A, B, lev, -1) == -brute.levenshtein(A, B)
        assert oracle.score(A, B, lcs, 0) == brute.lcs_length(A, B)


# ---------------------------------------------------------------- bulk entry points

def test_triangle_pairs_topk_query_agree_with_single_scores():
    v = zipf_vocab(60, seed=9, max_len=12)
    sim = oracle.sim_matrix(40, 1, -1)
    n = v.n
    tri = oracle.triangle(v.symbols, v.offsets, sim, -1, threads=3)
    assert tri.shape[0] == n * (n - 1) // 2
    idx = 0
    for i in range(n):
        for j in range(i + 1, n):
            assert tri[idx] == oracle.score(v.word(i), v.word(j), sim, -1)
            idx += 1
    # a sub-range of the triangle is the same slice
    part = oracle.triangle(v.symbols, v.offsets, sim, -1, 100, 777, threads=2)
    assert np.array_equal(part, tri[100:777])
    # explicit pair list
    pi = np.array([0, 5, 59, 3]); pj = np.array([1, 2, 0, 3])
    got = oracle.pairs(v.symbols, v.offsets, sim, -1, pi, pj)
    assert [int(x) for x in got] == [oracle.score(v.word(a), v.word(b), sim, -1) for a, b in zip(pi, pj)]
    # top-k by a full sort of a dense matrix built from single scores
    full = np.full((n, n), np.iinfo(np.int32).min, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            if i != j:
                full[i, j] = oracle.score(v.word(i), v.word(j), sim, -1)
    k = 7
    sc, ix, hist = oracle.topk_rows(v.symbols, v.offsets, sim, -1, k, hist_range=(-12, 12))
    for i in range(n):
        order = sorted((j for j in range(n) if j != i), key=lambda j: (-full[i, j], j))[:k]
        assert list(ix[i]) == order
        assert list(sc[i]) == [full[i, j] for j in order]
    assert int(hist.sum()) == n * (n - 1) // 2
    vals, counts = np.unique(tri, return_counts=True)
    for s, c in zip(vals, counts):
        assert hist[s + 12] == c
    # k larger than n-1 pads with (INT16_MIN, -1)
    sc2, ix2, _ = oracle.topk_rows(v.symbols, v.offsets, sim, -1, n + 3, r0=4, r1=6)
    assert list(ix2[0, n - 1:]) == [-1] * 4 and list(sc2[0, n - 1:]) == [-32768] * 4
    # query: no self exclusion, same key
    q = v.subset([3, 10])
    qs, qi = oracle.query(v.symbols, v.offsets, sim, -1, q.symbols, q.offsets, 5)
    for t, i in enumerate([3, 10]):
        row = [(oracle.score(v.word(i), v.word(j), sim, -1), j) for j in range(n)]
        row.sort(key=lambda x: (-x[0], x[1]))
        assert list(qi[t]) == [j for _, j in row[:5]]
        assert qi[t][0] == i and qs[t][0] == len(v.word(i))


def test_duplicate_words_are_distinct_neighbours():
    words = [[1, 2, 3], [1, 2, 3], [1, 2, 3], [4]]
    from synth import vocab_from_words
    v = vocab_from_words(words, 8)
    sim = oracle.sim_matrix(8, 1, -1)
    sc, ix, _ = oracle.topk_rows(v.symbols, v.offsets, sim, -1, 3)
    assert list(ix[1]) == [0, 2, 3] and list(sc[1]) == [3, 3, -3]


def test_uniform_vocab_with_submatrix_bounds():
    v = uniform_vocab(30, seed=3, alphabet=64, min_len=1, max_len=48)
    sub = random_submat(64, seed=4)
    sim = oracle.sim_matrix(64, submat=sub)
    lo, hi = oracle.score_bounds(48, sim, -2)
    assert (lo, hi) == (-144, 144)
    tri = oracle.triangle(v.symbols, v.offsets, sim, -2)
    assert tri.min() >= lo and tri.max() <= hi
