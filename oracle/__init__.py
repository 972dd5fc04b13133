"""CPU oracle for all-pairs Needleman-Wunsch scoring.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this package; the product library never does.  It
shares no code with the GPU path (it does not import the product package and
the product package does not import it).

Contents
--------
* ``nw_oracle.c`` (built into ``liboracle.so`` with gcc): Algorithm 1 of the
  paper literally, the row-major upper triangle, per-word top-k by full sort,
  per-query top-k, and the histogram of unordered-pair scores.
* :func:`edges`: the pairs whose raw score or normalised weight (Section 5)
  lies in a closed slice, filtered from the triangle in row-major order.
* ``brute.py``: the plain definition of the score (maximum over every global
  alignment), an explicit-alignment scorer, Levenshtein distance and LCS length.
* ``index_map.py``: the paper's row-major pair index and its inverse
  (Section 4.2, "Row & Column").

Scoring is given either as (match, mismatch, gap) or as a full similarity
matrix plus gap; :func:`sim_matrix` turns both into the int32 matrix the C code
reads, ``sim[x, y]`` = similarity of symbol x of word A with symbol y of word B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nw_oracle.c")
# NW_ORACLE_LIB names another build of the same source (the sanitizer build of
# the CPU tests); by default oracle/liboracle.so
_LIB = os.environ.get("NW_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/liboracle.so (or NW_ORACLE_LIB)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        flags = ["-O2"]
        if _LIB == _SAN_LIB:
            flags = _SAN_FLAGS
        subprocess.check_call(["gcc"] + flags + ["-std=c11", "-fPIC", "-shared", "-pthread",
                                                 "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


# AddressSanitizer + UndefinedBehaviorSanitizer, every report fatal.
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build_sanitized() -> str:
    """Compile the C oracle with AddressSanitizer and UBSan into oracle/liboracle_san.so.

    A process loads it with the sanitizer runtime preloaded
    (LD_PRELOAD=$(gcc -print-file-name=libasan.so)) and NW_ORACLE_LIB set to
    the returned path."""
    if not os.path.exists(_SAN_LIB) or os.path.getmtime(_SAN_LIB) < os.path.getmtime(_SRC):
        tmp = _SAN_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + _SAN_FLAGS + ["-std=c11", "-fPIC", "-shared", "-pthread",
                                                      "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _SAN_LIB)
    return _SAN_LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    lib.orc_score1.restype = i32
    lib.orc_score1.argtypes = [P, i64, P, i64, P, i32, i32]
    lib.orc_matrix.restype = None
    lib.orc_matrix.argtypes = [P, i64, P, i64, P, i32, i32, P]
    lib.orc_triangle.restype = ctypes.c_int
    lib.orc_triangle.argtypes = [P, P, i64, P, i32, i32, u64, u64, P, ctypes.c_int]
    lib.orc_pairs.restype = ctypes.c_int
    lib.orc_pairs.argtypes = [P, P, i64, P, i32, i32, P, P, i64, P, ctypes.c_int]
    lib.orc_topk_rows.restype = ctypes.c_int
    lib.orc_topk_rows.argtypes = [P, P, i64, P, i32, i32, i32, i64, i64, P, P, P, i32, i32,
                                  ctypes.c_int]
    lib.orc_query.restype = ctypes.c_int
    lib.orc_query.argtypes = [P, P, i64, P, i32, i32, P, P, i64, i32, P, P, ctypes.c_int]
    _lib = lib
    return lib


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def sim_matrix(alphabet: int, match: int = 1, mismatch: int = -1, submat=None) -> np.ndarray:
    """The similarity function of Algorithm 1 as a full int32 matrix."""
    if submat is not None:
        m = np.asarray(submat, dtype=np.int32)
        assert m.shape == (alphabet, alphabet)
        return np.ascontiguousarray(m)
    m = np.full((alphabet, alphabet), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return m


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def score(A, B, sim: np.ndarray, gap: int) -> int:
    """Algorithm 1 for one pair; A indexes the rows of the score matrix."""
    lib = _load()
    A = _c(A, np.uint8); B = _c(B, np.uint8); sim = _c(sim, np.int32)
    return int(lib.orc_score1(_p(A), A.shape[0], _p(B), B.shape[0], _p(sim), sim.shape[0], gap))


def matrix(A, B, sim: np.ndarray, gap: int) -> np.ndarray:
    """The full (len(A)+1) x (len(B)+1) score matrix of Algorithm 1."""
    lib = _load()
    A = _c(A, np.uint8); B = _c(B, np.uint8); sim = _c(sim, np.int32)
    M = np.zeros((A.shape[0] + 1, B.shape[0] + 1), dtype=np.int32)
    lib.orc_matrix(_p(A), A.shape[0], _p(B), B.shape[0], _p(sim), sim.shape[0], gap, _p(M))
    return M


def num_pairs(n: int) -> int:
    """E = n(n-1)/2 (Section 4.2, number of edges)."""
    return n * (n - 1) // 2


def triangle(symbols, offsets, sim, gap, idx_begin=0, idx_end=None, threads=None) -> np.ndarray:
    """int32 scores for pair indices [idx_begin, idx_end) of the row-major triangle."""
    lib = _load()
    symbols = _c(symbols, np.uint8); offsets = _c(offsets, np.uint64); sim = _c(sim, np.int32)
    n = offsets.shape[0] - 1
    E = num_pairs(n)
    if idx_end is None:
        idx_end = E
    assert 0 <= idx_begin <= idx_end <= E
    out = np.zeros(idx_end - idx_begin, dtype=np.int32)
    rc = lib.orc_triangle(_p(symbols), _p(offsets), n, _p(sim), sim.shape[0], gap,
                          idx_begin, idx_end, _p(out), threads or default_threads())
    assert rc == 0
    return out


def pairs(symbols, offsets, sim, gap, pi, pj, threads=None) -> np.ndarray:
    """int32 score(word pi[t], word pj[t]) for every t."""
    lib = _load()
    symbols = _c(symbols, np.uint8); offsets = _c(offsets, np.uint64); sim = _c(sim, np.int32)
    pi = _c(pi, np.int64); pj = _c(pj, np.int64)
    out = np.zeros(pi.shape[0], dtype=np.int32)
    rc = lib.orc_pairs(_p(symbols), _p(offsets), offsets.shape[0] - 1, _p(sim), sim.shape[0], gap,
                       _p(pi), _p(pj), pi.shape[0], _p(out), threads or default_threads())
    assert rc == 0
    return out


def topk_rows(symbols, offsets, sim, gap, k, r0=0, r1=None, hist_range=None, threads=None):
    """Per-word top-k for rows [r0, r1): (scores int32 [rows,k], index int32 [rows,k], hist).

    ``hist_range=(lo, hi)`` also returns the uint64 histogram of scores of the
    unordered pairs (i, j), j > i, whose row i lies in [r0, r1).
    """
    lib = _load()
    symbols = _c(symbols, np.uint8); offsets = _c(offsets, np.uint64); sim = _c(sim, np.int32)
    n = offsets.shape[0] - 1
    if r1 is None:
        r1 = n
    rows = r1 - r0
    sc = np.zeros((rows, k), dtype=np.int32)
    ix = np.zeros((rows, k), dtype=np.int32)
    hist = None
    hp, lo, nb = None, 0, 0
    if hist_range is not None:
        lo, hi = hist_range
        nb = hi - lo + 1
        hist = np.zeros(nb, dtype=np.uint64)
        hp = _p(hist)
    rc = lib.orc_topk_rows(_p(symbols), _p(offsets), n, _p(sim), sim.shape[0], gap, k, r0, r1,
                           _p(sc), _p(ix), hp, lo, nb, threads or default_threads())
    assert rc == 0
    return sc, ix, hist


def query(symbols, offsets, sim, gap, qsymbols, qoffsets, k, threads=None):
    """Per-query top-k over the whole dictionary: (scores int32 [nq,k], index int32 [nq,k])."""
    lib = _load()
    symbols = _c(symbols, np.uint8); offsets = _c(offsets, np.uint64); sim = _c(sim, np.int32)
    qsymbols = _c(qsymbols, np.uint8); qoffsets = _c(qoffsets, np.uint64)
    nq = qoffsets.shape[0] - 1
    sc = np.zeros((nq, k), dtype=np.int32)
    ix = np.zeros((nq, k), dtype=np.int32)
    rc = lib.orc_query(_p(symbols), _p(offsets), offsets.shape[0] - 1, _p(sim), sim.shape[0], gap,
                       _p(qsymbols), _p(qoffsets), nq, k, _p(sc), _p(ix), threads or default_threads())
    assert rc == 0
    return sc, ix


def normalised_weight(s: int, la: int, lb: int):
    """Section 5's normalised edge weight, exactly: 100 * score / max(len A, len B)
    as a Fraction (a pair of two empty words, score 0, has weight 0)."""
    from fractions import Fraction
    return Fraction(100 * int(s), max(int(la), int(lb), 1))


def in_slice(s, la, lb, lo: int, hi: int, normalised: bool = False, den: int = 1) -> np.ndarray:
    """Which pairs lie in the closed slice: lo <= s <= hi (raw), or
    lo/den <= 100 s / max(la, lb, 1) <= hi/den (normalised), in exact integers."""
    s = np.asarray(s, dtype=np.int64)
    if not normalised:
        return (s >= lo) & (s <= hi)
    m = np.maximum(np.maximum(np.asarray(la, np.int64), np.asarray(lb, np.int64)), 1)
    w = 100 * s * int(den)
    return (w >= int(lo) * m) & (w <= int(hi) * m)


def edges(symbols, offsets, sim, gap, lo, hi, normalised=False, den=1, idx_begin=0, idx_end=None, threads=None):
    """Edges of the word graph whose weight lies in a closed slice (Section 5 slices
    the graph by raw or normalised weight): (i, j, score) for the pairs i < j of
    row-major indices [idx_begin, idx_end), in that order.  Small n only (it
    enumerates every pair index)."""
    offsets = _c(offsets, np.uint64)
    n = offsets.shape[0] - 1
    E = num_pairs(n)
    if idx_end is None:
        idx_end = E
    s = triangle(symbols, offsets, sim, gap, idx_begin, idx_end, threads).astype(np.int64)
    i, j = np.triu_indices(n, 1)            # row-major pair order (Section 4.1)
    i, j = i[idx_begin:idx_end], j[idx_begin:idx_end]
    lens = np.diff(offsets).astype(np.int64)
    keep = in_slice(s, lens[i], lens[j], lo, hi, normalised, den)
    return i[keep].astype(np.int64), j[keep].astype(np.int64), s[keep].astype(np.int32)


def score_bounds(max_len: int, sim: np.ndarray, gap: int):
    """Range every optimal score of words of length <= max_len lies in (gap <= 0).

    Floor: the alignment that pairs min(la, lb) symbols and gaps the rest
    scores >= max(la, lb) * min(min S, p), so the optimum is >= L * min(min S, p, 0).
    Ceiling: at most L aligned symbol pairs, each <= max S, and gaps add <= 0.
    """
    smin = int(np.min(sim)); smax = int(np.max(sim))
    lo = max_len * min(smin, gap, 0)
    hi = max_len * max(smax, 0)
    return lo, hi
