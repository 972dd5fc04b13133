"""Seeded synthetic inputs for the all-pairs Needleman-Wunsch workloads.

This module only draws random data: symbol sequences, substitution matrices
and query arrival times.  It holds none of the alignment arithmetic, so both
the CPU oracle and the GPU path can take their inputs from it without sharing
any of the method's code.

The paper's own data (about 600k French words encoded as integer IPA symbol
IDs, Section 3) is not available; these laws stand in for it:

* symbols: a finite Zipf law, P(rank r) proportional to r**-s for r = 1..A,
  symbol id = r - 1, drawn i.i.d. per position;
* lengths: Poisson(mean) clamped (not resampled) into [lo, hi], or uniform;
* all lengths are drawn first, then all symbols in one call, from
  ``numpy.random.default_rng(seed)`` (PCG64).

A vocabulary is returned as ``(symbols uint8[sum L], offsets uint64[n+1])``:
word ``i`` is ``symbols[offsets[i]:offsets[i+1]]``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Vocab", "zipf_probs", "zipf_vocab", "uniform_vocab", "vocab_from_words",
    "random_submat", "poisson_arrivals", "plain_config", "batched_configs",
    "BATCHED_SIZES", "BATCHED_LMAX", "query_words", "sha256_vocab",
]


@dataclass
class Vocab:
    symbols: np.ndarray          # uint8 [sum L]
    offsets: np.ndarray          # uint64 [n+1]
    alphabet: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def word(self, i: int) -> np.ndarray:
        return self.symbols[int(self.offsets[i]):int(self.offsets[i + 1])]

    def words(self) -> list:
        return [self.word(i) for i in range(self.n)]

    def subset(self, idx) -> "Vocab":
        idx = np.asarray(idx, dtype=np.int64)
        return vocab_from_words([self.word(int(i)) for i in idx], self.alphabet)


def zipf_probs(alphabet: int, s: float) -> np.ndarray:
    r = np.arange(1, alphabet + 1, dtype=np.float64)
    p = r ** (-s)
    return p / p.sum()


def _pack(lengths: np.ndarray, symbols: np.ndarray, alphabet: int, meta: dict) -> Vocab:
    offsets = np.zeros(lengths.shape[0] + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    return Vocab(symbols.astype(np.uint8, copy=False), offsets, alphabet, meta)


def zipf_vocab(n: int, seed: int, alphabet: int = 40, zipf_s: float = 1.1,
               mean_len: float = 7.0, min_len: int = 1, max_len: int = 20) -> Vocab:
    """n words; lengths clip(Poisson(mean_len), min_len, max_len); Zipf symbols."""
    rng = np.random.default_rng(seed)
    lengths = np.clip(rng.poisson(mean_len, size=n), min_len, max_len).astype(np.int64)
    total = int(lengths.sum())
    symbols = rng.choice(alphabet, size=total, p=zipf_probs(alphabet, zipf_s))
    meta = dict(kind="zipf", n=n, seed=seed, alphabet=alphabet, zipf_s=zipf_s,
                mean_len=mean_len, min_len=min_len, max_len=max_len)
    return _pack(lengths, symbols, alphabet, meta)


def uniform_vocab(n: int, seed: int, alphabet: int, min_len: int, max_len: int) -> Vocab:
    """n words; lengths uniform in [min_len, max_len]; symbols uniform."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(min_len, max_len + 1, size=n).astype(np.int64)
    total = int(lengths.sum())
    symbols = rng.integers(0, alphabet, size=total)
    meta = dict(kind="uniform", n=n, seed=seed, alphabet=alphabet,
                min_len=min_len, max_len=max_len)
    return _pack(lengths, symbols, alphabet, meta)


def vocab_from_words(words, alphabet: int) -> Vocab:
    words = [np.asarray(w, dtype=np.uint8) for w in words]
    lengths = np.array([w.shape[0] for w in words], dtype=np.int64)
    symbols = np.concatenate(words) if words and lengths.sum() > 0 else np.zeros(0, np.uint8)
    return _pack(lengths, symbols, alphabet, dict(kind="explicit", n=len(words)))


def random_submat(alphabet: int, seed: int, lo: int = -3, hi: int = 3, diag: int = 3) -> np.ndarray:
    """Symmetric int8 matrix: strict upper triangle uniform in [lo, hi], mirrored, fixed diagonal."""
    rng = np.random.default_rng(seed)
    m = np.zeros((alphabet, alphabet), dtype=np.int8)
    iu = np.triu_indices(alphabet, k=1)
    m[iu] = rng.integers(lo, hi + 1, size=iu[0].shape[0])
    m = m + m.T
    np.fill_diagonal(m, diag)
    return m.astype(np.int8)


def poisson_arrivals(rate_qps: float, count: int, seed: int) -> np.ndarray:
    """Open-loop Poisson process: cumulative exponential gaps, seconds from t=0."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_qps, size=count))


# ---------------------------------------------------------------------------
# The workloads (sizes and laws of the benchmark configurations)
# ---------------------------------------------------------------------------

def plain_config(which: str) -> Vocab:
    """'small': 2,000 words; 'mid': 50,000 words; 'paper': 600,000 words.

    small/mid: 40-symbol Zipf(1.1), clip(Poisson(7), 1, 20);
    paper:     40-symbol Zipf(1.1), clip(Poisson(8), 1, 32).
    """
    if which == "small":
        return zipf_vocab(2000, seed=1, mean_len=7.0, max_len=20)
    if which == "mid":
        return zipf_vocab(50000, seed=2, mean_len=7.0, max_len=20)
    if which == "paper":
        return zipf_vocab(600000, seed=3, mean_len=8.0, max_len=32)
    raise ValueError(which)


BATCHED_SIZES = (1000, 3000, 10000, 20000, 40000, 60000, 80000, 100000)
# round(8 + 40 v / 7) for v = 0..7
BATCHED_LMAX = tuple(int(round(8 + 40 * v / 7)) for v in range(8))


def batched_configs(scale: float = 1.0):
    """Eight vocabularies (64-symbol uniform alphabet, uniform lengths 1..Lmax_v)
    and one seeded symmetric 64x64 substitution matrix in [-3, 3], diagonal +3.

    ``scale`` shrinks every vocabulary (for tests); sizes stay >= 2.
    """
    vocabs = []
    for v, (n, lmax) in enumerate(zip(BATCHED_SIZES, BATCHED_LMAX)):
        nv = max(2, int(round(n * scale)))
        vocabs.append(uniform_vocab(nv, seed=40 + v, alphabet=64, min_len=1, max_len=lmax))
    return vocabs, random_submat(64, seed=4)


def query_words(count: int, seed: int) -> Vocab:
    """Query words drawn like the 600k dictionary (Zipf-40, clip(Poisson(8), 1, 32))."""
    return zipf_vocab(count, seed=seed, mean_len=8.0, max_len=32)


def sha256_vocab(v: Vocab) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(v.offsets).tobytes())
    h.update(np.ascontiguousarray(v.symbols).tobytes())
    return h.hexdigest()
