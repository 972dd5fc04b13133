"""GPU parity of the fused all-pairs top-k and histogram against the oracle (bit-exact)."""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _gpu_topk(v, k, scoring=None, submat=None, gap=-1):
    import paper_2509_01654_amd as nw
    sc = nw.Scoring(v.alphabet, submat=submat, gap=gap, **(scoring or {}))
    dv = nw.Vocab(v.symbols, v.offsets, sc)
    s, i, h = dv.all_pairs_topk(k)
    torch.cuda.synchronize()
    return dv, s.cpu().numpy().astype(np.int32), i.cpu().numpy(), h.cpu().numpy().astype(np.uint64)


def _sim(v, submat=None, scoring=None):
    scoring = scoring or {}
    return oracle.sim_matrix(v.alphabet, scoring.get("match", 1), scoring.get("mismatch", -1), submat)


def test_small_config_top32_and_histogram():
    _report("small config top-32")
    v = synth.plain_config("small")
    dv, s, i, h = _gpu_topk(v, 32)
    lo, hi = dv.bounds
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, _sim(v), -1, 32, hist_range=(lo, hi))
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
    np.testing.assert_array_equal(h, wh)
    assert int(h.sum()) == v.n * (v.n - 1) // 2


@pytest.mark.parametrize("n,k", [(1, 4), (2, 1), (5, 8), (33, 32), (40, 32), (300, 63), (257, 1)])
def test_tiny_and_padding(n, k):
    _report(f"tiny n={n} k={k}")
    v = synth.zipf_vocab(n, seed=300 + n, mean_len=8.0, max_len=32)
    dv, s, i, h = _gpu_topk(v, k)
    lo, hi = dv.bounds
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, _sim(v), -1, k, hist_range=(lo, hi))
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
    np.testing.assert_array_equal(h, wh)


def test_heavy_ties_duplicates():
    """Two-symbol alphabet, lengths 0..3: thousands of identical words and tied scores."""
    _report("heavy ties")
    rng = np.random.default_rng(3)
    words = [rng.integers(0, 2, size=rng.integers(0, 4)) for _ in range(3000)]
    v = synth.vocab_from_words(words, 2)
    dv, s, i, h = _gpu_topk(v, 32)
    lo, hi = dv.bounds
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, _sim(v), -1, 32, hist_range=(lo, hi))
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
    np.testing.assert_array_equal(h, wh)


def test_submatrix_top16():
    _report("submatrix top-16")
    v = synth.uniform_vocab(2500, seed=45, alphabet=64, min_len=1, max_len=48)
    S = synth.random_submat(64, seed=4)
    dv, s, i, h = _gpu_topk(v, 16, submat=S, gap=-2)
    lo, hi = dv.bounds
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, _sim(v, S), -2, 16, hist_range=(lo, hi))
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
    np.testing.assert_array_equal(h, wh)


def test_probe_thresholds_sampled_rows():
    """20,000 words: the probe subset is a strict subset; sampled rows against the
    oracle's full sort, histogram against the oracle triangle's counts."""
    _report("n=20000 probes")
    v = synth.zipf_vocab(20000, seed=22, mean_len=8.0, max_len=32)
    dv, s, i, h = _gpu_topk(v, 32)
    lo, hi = dv.bounds
    rows = np.unique(np.concatenate([np.arange(0, 20), np.arange(9990, 10010), np.arange(19980, 20000),
                                     np.random.default_rng(1).integers(0, 20000, 140)]))
    for r in rows:
        ws, wi, _ = oracle.topk_rows(v.symbols, v.offsets, _sim(v), -1, 32, r0=int(r), r1=int(r) + 1)
        np.testing.assert_array_equal(i[r], wi[0])
        np.testing.assert_array_equal(s[r], ws[0])
    assert int(h.sum()) == v.n * (v.n - 1) // 2
    tri = oracle.triangle(v.symbols, v.offsets, _sim(v), -1)
    np.testing.assert_array_equal(h, np.bincount(tri - lo, minlength=hi - lo + 1).astype(np.uint64))


def test_overflow_recomputation(monkeypatch):
    """A tiny candidate capacity forces the exact recomputation of overflowed words."""
    _report("overflow recomputation")
    monkeypatch.setenv("NW_TOPK_CAP", "40")
    v = synth.zipf_vocab(17000, seed=23, mean_len=4.0, max_len=12)
    dv, s, i, h = _gpu_topk(v, 32)
    assert dv.topk_overflow_words() > 1000   # most words overflow a 40-key list
    rows = np.unique(np.concatenate([np.arange(0, 30), np.random.default_rng(2).integers(0, v.n, 100)]))
    for r in rows:
        ws, wi, _ = oracle.topk_rows(v.symbols, v.offsets, _sim(v), -1, 32, r0=int(r), r1=int(r) + 1)
        np.testing.assert_array_equal(i[r], wi[0])
        np.testing.assert_array_equal(s[r], ws[0])
