"""GPU parity of per-query top-k neighbour lists against the oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _run(v, q, k, submat=None, gap=-1):
    import paper_2509_01654_amd as nw
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, submat=submat, gap=gap))
    s, i = dv.query(q.symbols, q.offsets, k)
    torch.cuda.synchronize()
    sim = oracle.sim_matrix(v.alphabet, 1, -1, submat)
    ws, wi = oracle.query(v.symbols, v.offsets, sim, gap, q.symbols, q.offsets, k)
    return s.cpu().numpy().astype(np.int32), i.cpu().numpy(), ws, wi


@pytest.mark.parametrize("nq,k", [(1, 16), (2, 1), (37, 16), (200, 16), (64, 64)])
def test_queries_against_dictionary(nq, k):
    _report(f"queries nq={nq} k={k}")
    v = synth.zipf_vocab(6000, seed=50, mean_len=8.0, max_len=32)
    q = synth.query_words(nq, seed=51 + nq)
    s, i, ws, wi = _run(v, q, k)
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)


def test_query_edge_words():
    _report("query edge words")
    v = synth.zipf_vocab(3000, seed=52, mean_len=8.0, max_len=32)
    words = [[], [0], list(v.word(5)), list(v.word(5)), [7] * 48, list(range(40)), [1, 2, 3]]
    q = synth.vocab_from_words(words, 40)
    s, i, ws, wi = _run(v, q, 16)
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
    assert i[2][0] == 5 or s[2][0] == len(v.word(5))


def test_query_small_dictionary_pads():
    _report("query small dictionary")
    v = synth.zipf_vocab(5, seed=53)
    q = synth.query_words(9, seed=54)
    s, i, ws, wi = _run(v, q, 16)
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
    assert (i[:, 5:] == -1).all()


def test_query_submatrix():
    _report("query submatrix")
    v = synth.uniform_vocab(4000, seed=55, alphabet=64, min_len=1, max_len=48)
    S = synth.random_submat(64, seed=4)
    q = synth.uniform_vocab(50, seed=56, alphabet=64, min_len=1, max_len=48)
    s, i, ws, wi = _run(v, q, 16, submat=S, gap=-2)
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s, ws)
