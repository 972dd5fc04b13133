"""Row-major upper-triangle pair index (Section 4.2, "Row & Column").

TEST INFRASTRUCTURE ONLY.

Pairs (r, c), r < c, of n words are numbered in row-major order
(0,1), (0,2), ..., (0,n-1), (1,2), ..., (n-2,n-1) (Section 4.1).  S_r is the
number of pairs up to the end of row r:

    S_r = (n-1)(r+1) - r(r+1)/2,      S_{-1} = 0,     E = S_{n-1} = n(n-1)/2.

Forward: idx(r, c) = S_{r-1} + (c - r - 1).
Inverse (the paper's closed form, evaluated in float64 as the paper does):
    z = n - 1/2,  r = floor(z - sqrt(z^2 - 2 idx)),  c = r + 1 + idx - S_{r-1}.
"""
from __future__ import annotations

import math


def S(n: int, r: int) -> int:
    """Pairs traversed up to the end of row r (S_{-1} = 0)."""
    return (n - 1) * (r + 1) - r * (r + 1) // 2


def num_pairs(n: int) -> int:
    return n * (n - 1) // 2


def pair_index(n: int, r: int, c: int) -> int:
    if not (0 <= r < c < n):
        raise ValueError("need 0 <= r < c < n")
    return S(n, r - 1) + (c - r - 1)


def pair_of_index(n: int, idx: int):
    """The paper's float64 inverse: (r, c) for 0 <= idx < n(n-1)/2."""
    if not (0 <= idx < num_pairs(n)):
        raise ValueError("idx out of range")
    z = n - 0.5
    r = int(math.floor(z - math.sqrt(z * z - 2.0 * idx)))
    c = r + 1 + idx - S(n, r - 1)
    return r, c


def enumerate_pairs(n: int):
    """The traversal itself: every (r, c) in row-major order."""
    for r in range(n):
        for c in range(r + 1, n):
            yield r, c


def capacity_words(num_edges: int) -> float:
    """Largest n whose triangle has num_edges entries: n = 1/2 + sqrt(1/4 + 2E)."""
    return 0.5 + math.sqrt(0.25 + 2.0 * num_edges)
