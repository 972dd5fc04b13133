"""GPU parity on both sides of the block-size rule for mid-size dictionaries.

Above 32,768 words, dictionaries of words up to 24 symbols are cut into
2048-word blocks and those with longer words into 1024-word blocks (up to
131,072 words).  Whole triangles and top-k lists of 32,769-word dictionaries
of each kind against the oracle, bit-exact.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.mark.parametrize("max_len,mean_len", [(20, 7.0), (30, 12.0)])
def test_block_rule_triangle_and_topk(max_len, mean_len):
    import paper_2509_01654_amd as nw
    _report(f"32,769 words, lengths up to {max_len}: triangle and top-16")
    v = synth.zipf_vocab(32769, seed=90 + max_len, mean_len=mean_len, max_len=max_len)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, 1, -1, -1))
    sim = oracle.sim_matrix(v.alphabet, 1, -1)
    got = dv.all_pairs_scores(dtype=torch.int8)
    torch.cuda.synchronize()
    want = oracle.triangle(v.symbols, v.offsets, sim, -1)
    np.testing.assert_array_equal(got.cpu().numpy().astype(np.int32), want)
    s, i, h = dv.all_pairs_topk(16)
    torch.cuda.synchronize()
    lo, hi = dv.bounds
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, sim, -1, 16, hist_range=(lo, hi))
    np.testing.assert_array_equal(i.cpu().numpy(), wi)
    np.testing.assert_array_equal(s.cpu().numpy().astype(np.int32), ws)
    np.testing.assert_array_equal(h.cpu().numpy().astype(np.uint64), wh)
