"""The intra-pair anti-diagonal kernel (long words up to 255 symbols) against the oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _run(v, fn, dtype=torch.int16, submat=None, gap=-1, **kw):
    import paper_2509_01654_amd as nw
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, submat=submat, gap=gap, **kw))
    out = getattr(dv, fn)(dtype=dtype)
    torch.cuda.synchronize()
    return dv, out.cpu().numpy().astype(np.int32)


@pytest.mark.parametrize("maxlen", [64, 100, 160, 255])
def test_long_words_pm1(maxlen):
    _report(f"long words up to {maxlen}")
    v = synth.uniform_vocab(300, seed=70 + maxlen, alphabet=20, min_len=1, max_len=maxlen)
    _, got = _run(v, "all_pairs_scores")
    want = oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(20, 1, -1), -1)
    np.testing.assert_array_equal(got, want)


def test_long_words_submatrix_and_edges():
    _report("long words submatrix + edges")
    rng = np.random.default_rng(75)
    words = [[], [3], [7] * 255, [7] * 254, list(rng.integers(0, 64, 200)), list(rng.integers(0, 64, 49))]
    words += [list(rng.integers(0, 64, int(rng.integers(0, 256)))) for _ in range(120)]
    v = synth.vocab_from_words(words, 64)
    S = synth.random_submat(64, seed=4)
    _, got = _run(v, "all_pairs_scores", submat=S, gap=-2)
    want = oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(64, submat=S), -2)
    np.testing.assert_array_equal(got, want)
    _, naive = _run(v, "all_pairs_scores_naive", submat=S, gap=-2)
    np.testing.assert_array_equal(naive, want)


@pytest.mark.parametrize("n", [255, 1500])
def test_forced_diag_on_short_words(n):
    """The anti-diagonal path on a dictionary the register-row kernel also takes."""
    _report(f"forced anti-diagonal n={n}")
    v = synth.uniform_vocab(n, seed=76, alphabet=64, min_len=1, max_len=48)
    S = synth.random_submat(64, seed=4)
    _, got = _run(v, "all_pairs_scores_diag", submat=S, gap=-2)
    want = oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(64, submat=S), -2)
    np.testing.assert_array_equal(got, want)


def test_long_dictionary_refused_by_register_row_calls():
    import paper_2509_01654_amd as nw
    _report("long dictionary refused by top-k / query")
    v = synth.uniform_vocab(50, seed=77, alphabet=20, min_len=40, max_len=80)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(20, 1, -1, -1))
    with pytest.raises(nw.NwError):
        dv.all_pairs_topk(4)
    with pytest.raises(nw.NwError):
        dv.query(v.symbols[:5], np.array([0, 5], np.uint64), 4)


@pytest.mark.parametrize("alphabet", [120, 250])
def test_long_words_large_alphabets(alphabet):
    """Long words over large alphabets: 120 symbols still fit the longest class's
    profile in LDS; 250 do not and the call goes through the one-thread-per-pair
    kernel.  Triangle and threshold edges against the oracle."""
    import paper_2509_01654_amd as nw
    _report(f"long words, alphabet {alphabet}")
    v = synth.uniform_vocab(160, seed=80 + alphabet, alphabet=alphabet, min_len=150, max_len=255)
    sim = oracle.sim_matrix(alphabet, 1, -1)
    _, got = _run(v, "all_pairs_scores")
    want = oracle.triangle(v.symbols, v.offsets, sim, -1)
    np.testing.assert_array_equal(got, want)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(alphabet, 1, -1, -1))
    i, j, s, count = dv.all_pairs_edges(-95, -88, normalised=True)
    torch.cuda.synchronize()
    wi, wj, ws = oracle.edges(v.symbols, v.offsets, sim, -1, -95, -88, True)
    assert count == len(wi) > 1000
    key = lambda a, b: np.asarray(a, np.int64) * v.n + np.asarray(b, np.int64)  # noqa: E731
    k_got = key(i.cpu().numpy()[:count], j.cpu().numpy()[:count])
    order = np.argsort(k_got)
    np.testing.assert_array_equal(k_got[order], np.sort(key(wi, wj)))
    np.testing.assert_array_equal(s.cpu().numpy()[:count][order].astype(np.int32),
                                  np.asarray(ws, np.int32)[np.argsort(key(wi, wj))])


@pytest.mark.parametrize("fn", ["all_pairs_scores", "all_pairs_scores_diag"])
def test_long_words_index_ranges(fn):
    """Sub-ranges of the triangle (ragged starts and ends inside rows and
    blocks) through the anti-diagonal kernel."""
    import paper_2509_01654_amd as nw
    _report(f"long words index ranges ({fn})")
    v = synth.uniform_vocab(700, seed=83, alphabet=30, min_len=1, max_len=220)
    sim = oracle.sim_matrix(30, 2, -1)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(30, 2, -1, -2))
    E = dv.num_pairs
    for b0, b1 in ((0, 1), (E - 1, E), (1234, 1234 + 70_001), (E // 3 - 17, E // 3 + 5), (100, E - 100)):
        got = getattr(dv, fn)(b0, b1, dtype=torch.int16)
        torch.cuda.synchronize()
        want = oracle.triangle(v.symbols, v.offsets, sim, -2, b0, b1)
        np.testing.assert_array_equal(got.cpu().numpy().astype(np.int32), want, err_msg=f"[{b0}, {b1})")
