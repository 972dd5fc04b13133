"""GPU parity of the threshold edge emitter (raw and normalised weight slices,
Section 5) against the CPU oracle.  The edges come back in no particular
order: the sets are compared exactly, and the stored subset of a truncated
call is checked for validity.  Every case prints its name before the GPU work.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PM1 = dict(match=1, mismatch=-1, gap=-1)


def _nw():
    import paper_2509_01654_amd as nw
    return nw


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _vocab(v, submat=None, **kw):
    nw = _nw()
    return nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, submat=submat, **kw))


def _sorted(i, j, s, n):
    i = np.asarray(i, np.int64); j = np.asarray(j, np.int64); s = np.asarray(s, np.int32)
    order = np.argsort(i * max(n, 1) + j, kind="stable")
    return i[order], j[order], s[order]


def _gpu_edges(dv, *a, **kw):
    i, j, s, count = dv.all_pairs_edges(*a, **kw)
    return i.cpu().numpy(), j.cpu().numpy(), s.cpu().numpy(), count


def _check_equal(got, want, n):
    gi, gj, gs = _sorted(*got, n)
    wi, wj, ws = want
    np.testing.assert_array_equal(gi, wi)
    np.testing.assert_array_equal(gj, wj)
    np.testing.assert_array_equal(gs, ws)


SMALL_SLICES = [
    ("raw [-3,1]", False, -3, 1, 1),
    ("raw [5,20]", False, 5, 20, 1),
    ("raw one bin", False, -7, -7, 1),
    ("norm [60,100]", True, 60, 100, 1),
    ("norm [40,49]", True, 40, 49, 1),
    ("norm [8,10]", True, 8, 10, 1),
    ("norm 200/3", True, 200, 200, 3),
    ("norm [-100,-100]", True, -100, -100, 1),
    ("norm beyond max", True, 101, 1000, 1),
]


@pytest.mark.parametrize("name,normalised,lo,hi,den", SMALL_SLICES)
def test_small_config_slices(name, normalised, lo, hi, den):
    """2,000 Zipf-40 words, +1/-1/-1: the edge set of each slice equals the oracle's."""
    _report(f"edges small config {name}")
    v = synth.plain_config("small")
    sim = oracle.sim_matrix(40, 1, -1)
    dv = _vocab(v, **PM1)
    i, j, s, count = _gpu_edges(dv, lo, hi, normalised, den)
    want = oracle.edges(v.symbols, v.offsets, sim, -1, lo, hi, normalised, den)
    assert count == len(want[0]) == len(i)
    _check_equal((i, j, s), want, v.n)


def test_whole_range_is_the_triangle():
    _report("edges whole score range = triangle")
    v = synth.plain_config("small")
    dv = _vocab(v, **PM1)
    lo, hi = dv.bounds
    i, j, s, count = _gpu_edges(dv, lo, hi)
    assert count == dv.num_pairs
    gi, gj, gs = _sorted(i, j, s, v.n)
    tri = oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1)
    ti, tj = np.triu_indices(v.n, 1)
    np.testing.assert_array_equal(gi, ti)
    np.testing.assert_array_equal(gj, tj)
    np.testing.assert_array_equal(gs, tri)


def test_index_range_chunks():
    """Ragged [idx_begin, idx_end) chunks: each equals the oracle's chunk, together the whole set."""
    _report("edges index-range chunks")
    v = synth.plain_config("small")
    sim = oracle.sim_matrix(40, 1, -1)
    dv = _vocab(v, **PM1)
    E = dv.num_pairs
    cuts = [0, 1, 777_777, 777_778, 1_500_001, E]
    parts = []
    for b0, b1 in zip(cuts[:-1], cuts[1:]):
        got = _gpu_edges(dv, 30, 100, True, 1, idx_begin=b0, idx_end=b1)
        want = oracle.edges(v.symbols, v.offsets, sim, -1, 30, 100, True, 1, b0, b1)
        assert got[3] == len(want[0])
        _check_equal(got[:3], want, v.n)
        parts.append(want)
    full = oracle.edges(v.symbols, v.offsets, sim, -1, 30, 100, True, 1)
    assert sum(len(p[0]) for p in parts) == len(full[0])


def test_truncation_and_count_only():
    """cap below the count: the count stays exact, the stored edges are distinct true edges."""
    _report("edges truncation + count only")
    v = synth.plain_config("small")
    sim = oracle.sim_matrix(40, 1, -1)
    dv = _vocab(v, **PM1)
    wi, wj, ws = oracle.edges(v.symbols, v.offsets, sim, -1, -2, 2)
    total = len(wi)
    truth = dict(zip((wi * v.n + wj).tolist(), ws.tolist()))
    for cap in (0, 1, 63, total // 3, total - 1, total, total + 5):
        i, j, s, count = _gpu_edges(dv, -2, 2, cap=cap)
        assert count == total
        assert len(i) == min(cap, total)
        keys = i.astype(np.int64) * v.n + j
        assert len(np.unique(keys)) == len(keys)
        assert all(truth.get(k) == sc for k, sc in zip(keys.tolist(), s.tolist()))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 257, 700])
def test_ragged_and_degenerate_sizes(n):
    _report(f"edges ragged n={n}")
    v = synth.zipf_vocab(n, seed=2000 + n, mean_len=8.0, max_len=32)
    dv = _vocab(v, **PM1)
    i, j, s, count = _gpu_edges(dv, -5, 100, True, 1)
    want = oracle.edges(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, -5, 100, True, 1)
    assert count == len(want[0])
    _check_equal((i, j, s), want, n)


def test_batched_vocabulary_submatrix():
    """A 64-symbol dictionary with the seeded similarity matrix and gap -2, words up to 48."""
    _report("edges submatrix vocabulary")
    v = synth.uniform_vocab(1500, seed=41, alphabet=64, min_len=1, max_len=48)
    S = synth.random_submat(64, seed=4)
    sim = oracle.sim_matrix(64, submat=S)
    dv = _vocab(v, submat=S, gap=-2)
    for lo, hi, norm in ((0, 100, True), (-20, -5, False)):
        got = _gpu_edges(dv, lo, hi, norm)
        want = oracle.edges(v.symbols, v.offsets, sim, -2, lo, hi, norm)
        assert got[3] == len(want[0])
        _check_equal(got[:3], want, v.n)


def test_long_words_take_the_anti_diagonal_kernel():
    _report("edges long words")
    rng = np.random.default_rng(91)
    words = [[], [2], [7] * 255, [7] * 200, list(rng.integers(0, 20, 120))]
    words += [list(rng.integers(0, 20, int(rng.integers(0, 256)))) for _ in range(200)]
    v = synth.vocab_from_words(words, 20)
    sim = oracle.sim_matrix(20, 1, -1)
    dv = _vocab(v, **PM1)
    assert dv.max_len > 48
    for lo, hi, norm in ((-30, 100, True), (-300, -100, False)):
        got = _gpu_edges(dv, lo, hi, norm)
        want = oracle.edges(v.symbols, v.offsets, sim, -1, lo, hi, norm)
        assert got[3] == len(want[0])
        _check_equal(got[:3], want, v.n)


def test_argument_errors():
    _report("edges argument errors")
    nw = _nw()
    v = synth.zipf_vocab(50, seed=3)
    dv = _vocab(v, **PM1)
    lib = nw.load_library()
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    sbuf = torch.zeros(64, dtype=torch.int16, device="cuda")
    P = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)  # noqa: E731

    def call(mode, lo, hi, den, b0=0, b1=None, cnt_off=0, cap=64):
        f = nw._EdgeFilter(mode, lo, hi, den)
        return lib.nw_all_pairs_edges(dv._h, b0, dv.num_pairs if b1 is None else b1, ctypes.byref(f), P(buf), P(buf),
                                      P(sbuf), cap, P(cnt, cnt_off), nw._stream_handle(None))

    assert call(2, 0, 1, 1) == nw.NW_EINVAL
    assert call(0, 2, 1, 1) == nw.NW_EINVAL
    assert call(1, 0, 1, 0) == nw.NW_EINVAL
    assert call(1, 0, 1, 1_000_001) == nw.NW_EINVAL
    assert call(0, 0, 1, 1, cnt_off=4) == nw.NW_EINVAL
    assert call(0, 0, 1, 1, b1=dv.num_pairs + 1) == nw.NW_EINVAL
    assert call(0, 0, 1, 1, b0=5, b1=4) == nw.NW_EINVAL
    assert call(0, 0, 1, 0) == nw.NW_OK          # den is ignored for raw slices
    torch.cuda.synchronize()
    S = synth.random_submat(40, seed=9)
    S[0, 1] = S[1, 0] + 1
    dva = _vocab(v, submat=S, gap=-1)
    f = nw._EdgeFilter(0, 0, 1, 1)
    assert lib.nw_all_pairs_edges(dva._h, 0, dva.num_pairs, ctypes.byref(f), P(buf), P(buf), P(sbuf), 64, P(cnt),
                                  nw._stream_handle(None)) == nw.NW_EINVAL


def test_full_size_paper_workload_sampled():
    """600,000 words: the normalised slice [60, 100] (the slice of the paper's ego
    networks).  Sampled edges are re-scored by the oracle; the raw-slice counts
    equal the histogram of the fused top-k pass; chunked calls add up."""
    _report("edges 600k paper workload")
    v = synth.plain_config("paper")
    sim = oracle.sim_matrix(40, 1, -1)
    dv = _vocab(v, **PM1)
    n = v.n
    i, j, s, count = dv.all_pairs_edges(60, 100, True, 1)
    assert count == i.numel() > 0
    keys = i.to(torch.int64) * n + j.to(torch.int64)
    assert torch.unique(keys).numel() == count
    assert bool((i < j).all()) and bool((i >= 0).all()) and bool((j < n).all())
    rng = np.random.default_rng(5)
    pick = rng.choice(count, size=min(count, 3000), replace=False)
    pi, pj, ps = i.cpu().numpy()[pick], j.cpu().numpy()[pick], s.cpu().numpy()[pick]
    np.testing.assert_array_equal(oracle.pairs(v.symbols, v.offsets, sim, -1, pi, pj), ps)
    lens = v.lengths.astype(np.int64)
    assert oracle.in_slice(ps, lens[pi], lens[pj], 60, 100, True, 1).all()
    # rows re-scored in full: every partner of a sampled row that passes is an edge
    rows = rng.choice(n, size=4, replace=False)
    ii, jj = i.cpu().numpy().astype(np.int64), j.cpu().numpy().astype(np.int64)
    for r in rows.tolist():
        others = np.arange(n, dtype=np.int64)
        others = others[others != r]
        sc = oracle.pairs(v.symbols, v.offsets, sim, -1, np.full(others.shape, r), others)
        ok = oracle.in_slice(sc, lens[r], lens[others], 60, 100, True, 1)
        want = set(others[ok].tolist())
        got = set(jj[ii == r].tolist()) | set(ii[jj == r].tolist())
        assert got == want, r
    del i, j, s, keys
    # raw slice counts against the histogram of the fused top-k pass
    _, _, hist = dv.all_pairs_topk(k=1, hist=True)
    hist = hist.cpu().numpy()
    lo, hi = dv.bounds          # every score lies in [lo, hi]
    for a, b in ((5, 32), (0, 0), (-32, -20)):
        _, _, _, c = dv.all_pairs_edges(a, b, cap=0)
        assert c == int(hist[max(a, lo) - lo:min(b, hi) - lo + 1].sum()), (a, b)
    # three chunks add up to the whole call
    E = dv.num_pairs
    cuts = [0, E // 3, 2 * E // 3 + 7, E]
    total = sum(dv.all_pairs_edges(60, 100, True, 1, cap=0, idx_begin=a, idx_end=b)[3]
                for a, b in zip(cuts[:-1], cuts[1:]))
    assert total == count
