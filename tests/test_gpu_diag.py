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
