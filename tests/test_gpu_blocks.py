"""GPU parity on both sides of the block-size rules.

Above 32,768 words, dictionaries of words up to 24 symbols are cut into
2048-word blocks and those with longer words into 1024-word blocks (up to
131,072 words); larger dictionaries into 3072-word blocks.  Whole triangles
and top-k lists of 32,769-word dictionaries of each kind against the oracle,
bit-exact; at 131,072 / 131,073 words, sampled triangle entries, whole rows
at the block boundaries and sampled top-16 rows against the oracle, and the
top-k histogram against the counts of the triangle.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import index_map

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


@pytest.mark.parametrize("n,max_len,mean_len,block", [(131072, 20, 7.0, 2048), (131073, 20, 7.0, 3072),
                                                       (131073, 30, 12.0, 3072)])
def test_large_block_rule_sampled(n, max_len, mean_len, block):
    import paper_2509_01654_amd as nw
    _report(f"{n:,} words, lengths up to {max_len} ({block}-word blocks): sampled triangle and top-16")
    v = synth.zipf_vocab(n, seed=130 + max_len + n % 2, mean_len=mean_len, max_len=max_len)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, 1, -1, -1))
    sim = oracle.sim_matrix(v.alphabet, 1, -1)
    E = dv.num_pairs
    out = dv.all_pairs_scores(dtype=torch.int8)
    torch.cuda.synchronize()
    # rows on both sides of every block boundary, plus random ones
    edges = np.arange(block, n - 1, block)
    rows_b = np.unique(np.concatenate([edges - 1, edges, [0, n - 2]]))
    rng = np.random.default_rng(n + max_len)
    idx = np.unique(np.concatenate([rng.integers(0, E, 1_000_000), np.arange(E - 50, E),
                                    [index_map.S(n, r - 1) for r in rows_b.tolist()]]))
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.int32)
    starts = np.array([index_map.S(n, r) for r in range(n - 1)], np.int64)
    rows = np.searchsorted(starts, idx, side="right")
    cols = rows + 1 + idx - np.array([index_map.S(n, r - 1) for r in rows.tolist()], np.int64)
    np.testing.assert_array_equal(got, oracle.pairs(v.symbols, v.offsets, sim, -1, rows, cols))
    for r in rows_b[:: max(1, len(rows_b) // 12)].tolist():
        b0, b1 = index_map.S(n, r - 1), index_map.S(n, r)
        np.testing.assert_array_equal(out[b0:b1].cpu().numpy().astype(np.int32),
                                      oracle.triangle(v.symbols, v.offsets, sim, -1, b0, b1), err_msg=f"row {r}")
    # the top-k histogram (its own kernels) against the counts of the triangle
    lo, hi = dv.bounds
    counts = torch.zeros(hi - lo + 1, dtype=torch.int64, device=out.device)
    for c0 in range(0, E, 1 << 30):
        counts += torch.bincount(out[c0:c0 + (1 << 30)].to(torch.int32) - lo, minlength=hi - lo + 1)
    del out
    s, i, h = dv.all_pairs_topk(16)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(h.cpu().numpy().astype(np.int64), counts.cpu().numpy())
    s, i = s.cpu().numpy().astype(np.int32), i.cpu().numpy()
    picks = np.unique(np.concatenate([rows_b, [n - 1], rng.integers(0, n, 120)]))
    for r in picks[:: max(1, len(picks) // 160)].tolist():
        ws, wi, _ = oracle.topk_rows(v.symbols, v.offsets, sim, -1, 16, r0=r, r1=r + 1)
        np.testing.assert_array_equal(i[r], wi[0], err_msg=f"row {r}")
        np.testing.assert_array_equal(s[r], ws[0], err_msg=f"row {r}")
