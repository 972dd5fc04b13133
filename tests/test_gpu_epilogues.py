"""GPU parity of both epilogue forms of the tiled kernels against the oracle.

The triangle and top-k kernels with score codes apply while every score code
fits the binary16 window they use (triangle scores in [-256, 768); top-k
score ranges below 1024 values and histograms of at most 256 bins); wider
scoring schemes take the kernels with the plain integer epilogue.  These
cases pin both sides of that switch, and the dword-wide triangle stores on
output buffers of every byte alignment.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _nw():
    import paper_2509_01654_amd as nw
    return nw


@pytest.fixture(scope="module")
def mid_words():
    # more than 16,384 words: one launch per row length (the tiled kernels)
    return synth.zipf_vocab(16500, seed=77, mean_len=7.0, max_len=20)


@pytest.fixture(scope="module")
def mid_oracle(mid_words):
    v = mid_words
    return oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(v.alphabet, 1, -1), -1)


@pytest.mark.parametrize("dtype,shift", [("int8", 1), ("int8", 2), ("int8", 3), ("int16", 1)])
def test_triangle_codes_any_alignment(mid_words, mid_oracle, dtype, shift):
    """Whole triangle into a buffer starting 1..3 bytes (or one int16) past an aligned address."""
    _report(f"triangle codes {dtype} shifted by {shift}")
    nw = _nw()
    v = mid_words
    dt = getattr(torch, dtype)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, 1, -1, -1))
    base = torch.full((dv.num_pairs + 8,), 99, dtype=dt, device="cuda")
    out = base[shift:shift + dv.num_pairs]
    dv.all_pairs_scores(dtype=dt, out=out)
    torch.cuda.synchronize()
    got = base.cpu().numpy().astype(np.int32)
    np.testing.assert_array_equal(got[shift:shift + dv.num_pairs], mid_oracle)
    # nothing written outside the range
    assert (got[:shift] == 99).all() and (got[shift + dv.num_pairs:] == 99).all()


@pytest.mark.parametrize("shift", [1, 3])
def test_triangle_codes_partial_rows(mid_words, mid_oracle, shift):
    """Index ranges that start and end inside rows, into shifted buffers."""
    _report(f"triangle codes partial rows shifted by {shift}")
    nw = _nw()
    v = mid_words
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, 1, -1, -1))
    for ib, ie in [(12345, 12345 + 70_000_001), (dv.num_pairs - 5_000_003, dv.num_pairs), (7, 8)]:
        base = torch.full((ie - ib + 8,), 99, dtype=torch.int8, device="cuda")
        out = base[shift:shift + ie - ib]
        dv.all_pairs_scores(ib, ie, dtype=torch.int8, out=out)
        torch.cuda.synchronize()
        got = base.cpu().numpy().astype(np.int32)
        np.testing.assert_array_equal(got[shift:shift + ie - ib], mid_oracle[ib:ie])
        assert (got[:shift] == 99).all() and (got[shift + ie - ib:] == 99).all()


def test_triangle_wide_scores_plain_epilogue():
    """Scores beyond [-256, 768): the plain triangle kernels."""
    _report("triangle wide scores")
    nw = _nw()
    v = synth.zipf_vocab(16500, seed=78, mean_len=6.0, max_len=16)
    sc = dict(match=40, mismatch=-30, gap=-1)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, **sc))
    lo, hi = dv.bounds
    assert lo < -256 or hi >= 768
    got = dv.all_pairs_scores(dtype=torch.int16)
    torch.cuda.synchronize()
    want = oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(v.alphabet, 40, -30), -1)
    np.testing.assert_array_equal(got.cpu().numpy().astype(np.int32), want)


@pytest.mark.parametrize("hist", [True, False])
def test_topk_both_epilogues(hist):
    """513 score values: with the histogram (513 bins) the plain kernels, without it the code kernels."""
    _report(f"top-k 513 score values hist={hist}")
    nw = _nw()
    v = synth.zipf_vocab(6000, seed=79, mean_len=8.0, max_len=32)
    sc = dict(match=8, mismatch=-8, gap=-1)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, **sc))
    lo, hi = dv.bounds
    assert 256 < hi - lo + 1 < 1024
    s, i, h = dv.all_pairs_topk(16, hist=hist)
    torch.cuda.synchronize()
    sim = oracle.sim_matrix(v.alphabet, 8, -8)
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, sim, -1, 16, hist_range=(lo, hi))
    np.testing.assert_array_equal(i.cpu().numpy(), wi)
    np.testing.assert_array_equal(s.cpu().numpy().astype(np.int32), ws)
    if hist:
        np.testing.assert_array_equal(h.cpu().numpy().astype(np.uint64), wh)


def test_topk_wide_scores_plain_epilogue():
    """Over 1024 score values: the plain top-k kernels."""
    _report("top-k wide scores")
    nw = _nw()
    v = synth.zipf_vocab(4000, seed=80, mean_len=8.0, max_len=32)
    sc = dict(match=40, mismatch=-40, gap=-1)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, **sc))
    lo, hi = dv.bounds
    assert hi - lo + 1 > 1024
    s, i, h = dv.all_pairs_topk(8)
    torch.cuda.synchronize()
    sim = oracle.sim_matrix(v.alphabet, 40, -40)
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, sim, -1, 8, hist_range=(lo, hi))
    np.testing.assert_array_equal(i.cpu().numpy(), wi)
    np.testing.assert_array_equal(s.cpu().numpy().astype(np.int32), ws)
    np.testing.assert_array_equal(h.cpu().numpy().astype(np.uint64), wh)
