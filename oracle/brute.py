"""Plain definitions the DP oracle is pinned against (small inputs only).

TEST INFRASTRUCTURE ONLY.

* :func:`alignments` enumerates every global alignment of two words: sequences
  of columns that are (symbol, symbol), (symbol, gap) or (gap, symbol), which
  consume both words completely.  Their number is the Delannoy number D(m, n).
* :func:`alignment_score` scores one explicit alignment: the sum of similarity
  values over aligned symbol pairs plus p per gap symbol (Section 2; leading and
  trailing gaps count, since the first row and column of the score matrix are
  p times the index).
* :func:`brute_score` is the maximum over all alignments -- the quantity the
  paper's Algorithm 1 returns by the principle of optimality (Section 2).
* :func:`levenshtein` and :func:`lcs_length` are the textbook edit distance and
  longest-common-subsequence length, written independently of Algorithm 1.
  With match 0 / mismatch -1 / gap -1 the NW score equals -levenshtein; with
  match 1 / mismatch 0 / gap 0 it equals the LCS length.
"""
from __future__ import annotations

from functools import lru_cache

GAP = None  # marker for a gap in an alignment column


def alignments(A, B):
    """Yield every global alignment of A and B as a tuple of (x, y) columns,
    where x is a symbol of A or GAP and y a symbol of B or GAP."""
    A = tuple(int(x) for x in A)
    B = tuple(int(y) for y in B)

    def rec(i, j):
        if i == len(A) and j == len(B):
            yield ()
            return
        if i < len(A) and j < len(B):
            for rest in rec(i + 1, j + 1):
                yield ((A[i], B[j]),) + rest
        if i < len(A):
            for rest in rec(i + 1, j):
                yield ((A[i], GAP),) + rest
        if j < len(B):
            for rest in rec(i, j + 1):
                yield ((GAP, B[j]),) + rest

    yield from rec(0, 0)


def alignment_score(columns, sim, gap: int) -> int:
    """Score of one explicit alignment: similarity per aligned pair, p per gap."""
    total = 0
    for x, y in columns:
        if x is GAP and y is GAP:
            raise ValueError("a column cannot hold two gaps")
        if x is GAP or y is GAP:
            total += gap
        else:
            total += int(sim[x][y])
    return total


def brute_score(A, B, sim, gap: int) -> int:
    """max over all global alignments of alignment_score (exponential)."""
    return max(alignment_score(c, sim, gap) for c in alignments(A, B))


def count_alignments(m: int, n: int) -> int:
    """Delannoy number D(m, n) by its recurrence (independent of the generator)."""
    @lru_cache(maxsize=None)
    def d(a, b):
        if a == 0 or b == 0:
            return 1
        return d(a - 1, b) + d(a, b - 1) + d(a - 1, b - 1)
    return d(m, n)


def levenshtein(A, B) -> int:
    """Minimum number of single-symbol insertions, deletions and substitutions."""
    A = list(A); B = list(B)
    prev = list(range(len(B) + 1))
    for i in range(1, len(A) + 1):
        cur = [i] + [0] * len(B)
        for j in range(1, len(B) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (0 if A[i - 1] == B[j - 1] else 1))
        prev = cur
    return prev[len(B)]


def lcs_length(A, B) -> int:
    """Length of a longest common subsequence."""
    A = list(A); B = list(B)
    prev = [0] * (len(B) + 1)
    for i in range(1, len(A) + 1):
        cur = [0] * (len(B) + 1)
        for j in range(1, len(B) + 1):
            cur[j] = prev[j - 1] + 1 if A[i - 1] == B[j - 1] else max(prev[j], cur[j - 1])
        prev = cur
    return prev[len(B)]
