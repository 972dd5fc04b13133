"""Parity at the full benchmark sizes, in the launch configurations the bench
times, on outputs the oracle can compute one by one: sampled rows of the
600,000-word top-32, sampled pairs of the 50,000-word triangle and of the
eight batched triangles, and served queries against the 600,000-word
dictionary.  Every case prints its name before the GPU work."""
import numpy as np
import pytest

import oracle
import synth
from oracle import index_map

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _nw():
    import paper_2509_01654_amd as nw
    return nw


def _pm1():
    return oracle.sim_matrix(40, 1, -1)


@pytest.fixture(scope="module")
def paper():
    nw = _nw()
    v = synth.plain_config("paper")
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    return v, dv


def _pairs_of(n, idx):
    ij = [index_map.pair_of_index(n, int(t)) for t in idx]
    return np.array([p[0] for p in ij], np.int64), np.array([p[1] for p in ij], np.int64)


def test_paper_top32_histogram_sampled_rows(paper):
    """600,000 words, k = 32 with the histogram (the bench step): sampled rows
    against the oracle's full sort over all 599,999 partners."""
    _report("full size: 600k top-32 + histogram")
    v, dv = paper
    n, k = v.n, 32
    sc, ix, h = dv.all_pairs_topk(k)
    torch.cuda.synchronize()
    assert dv.topk_overflow_words() == 0
    h = h.cpu().numpy()
    assert int(h.sum()) == n * (n - 1) // 2
    sc, ix = sc.cpu().numpy(), ix.cpu().numpy()
    # every list sorted by (score desc, index asc), no self-loops, indices valid
    assert (np.diff(sc.astype(np.int32), axis=1) <= 0).all()
    ties = np.diff(sc.astype(np.int32), axis=1) == 0
    assert (np.diff(ix.astype(np.int64), axis=1)[ties] > 0).all()
    assert (ix >= 0).all() and (ix < n).all() and (ix != np.arange(n)[:, None]).all()
    rng = np.random.default_rng(17)
    CB = 2048
    rows = np.unique(np.concatenate([np.arange(0, 6), np.arange(n - 6, n), [CB - 1, CB, 2 * CB - 1, 5 * CB + 7],
                                     rng.integers(0, n, 30)]))
    for r in rows:
        ws, wi, _ = oracle.topk_rows(v.symbols, v.offsets, _pm1(), -1, k, r0=int(r), r1=int(r) + 1)
        np.testing.assert_array_equal(ix[r], wi[0], err_msg=f"row {r}")
        np.testing.assert_array_equal(sc[r].astype(np.int32), ws[0], err_msg=f"row {r}")


def _fixture_module():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_topk600k.py")
    spec = importlib.util.spec_from_file_location("make_topk600k", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_paper_top32_every_row_against_fixture(paper):
    """600,000 words, k = 32: every row's list and every histogram bin against
    the oracle's run over all rows (stored as SHA-256 digests of 1,024-row
    blocks, tests/golden/topk600k_paper.txt), the byte-for-byte comparison of
    CPU and GPU outputs of Section 5."""
    import os
    fx = _fixture_module()
    if not os.path.exists(fx.FIXTURE):
        pytest.skip("the 600k oracle fixture has not been generated")
    want = fx.read_fixture()
    v, dv = paper
    assert want["dataset_sha256"] == synth.sha256_vocab(v), "the fixture belongs to another dataset"
    assert want["n"] == v.n and want["k"] == 32
    _report("full size: 600k top-32 every row against the oracle fixture")
    sc, ix, h = dv.all_pairs_topk(32)
    torch.cuda.synchronize()
    sc, ix, h = sc.cpu().numpy(), ix.cpu().numpy(), h.cpu().numpy().astype(np.uint64)
    # the fixture's bins cover -32 .. 32; the dictionary's own score range lies inside
    lo, hi = dv.bounds
    a, b = lo - want["hist_lo"], hi - want["hist_lo"] + 1
    assert 0 <= a and b <= len(want["hist"]) and len(h) == b - a
    np.testing.assert_array_equal(h, want["hist"][a:b], err_msg="histogram bins differ from the oracle")
    assert not want["hist"][:a].any() and not want["hist"][b:].any()
    B = want["block_rows"]
    bad = [blk for blk in range((v.n + B - 1) // B)
           if fx.block_digest(sc[blk * B:(blk + 1) * B], ix[blk * B:(blk + 1) * B]) != want["blocks"][blk]]
    assert not bad, f"{len(bad)} blocks of {B} rows differ from the oracle, first {bad[:8]}"


def test_mid_triangle_sampled_pairs():
    """50,000 words, the int8 triangle of the bench: a random sample of 10^6 pair
    indices, every block-boundary row start, the last pairs, and two full blocks
    of 100 rows (all their partners) against the oracle."""
    nw = _nw()
    _report("full size: 50k int8 triangle")
    v = synth.plain_config("mid")
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    out = dv.all_pairs_scores(dtype=torch.int8)
    torch.cuda.synchronize()
    n, E = v.n, dv.num_pairs
    rng = np.random.default_rng(3)
    starts = [index_map.S(n, r - 1) for r in range(0, n - 1, 1024)]
    idx = np.unique(np.concatenate([rng.integers(0, E, 1_000_000), starts, np.arange(E - 50, E), np.arange(0, 50)]))
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.int32)
    # rows from the integer row starts S_r (the index map pinned in test_index_map)
    rows = np.searchsorted(np.array([index_map.S(n, r) for r in range(n - 1)], np.int64), idx, side="right")
    cols = rows + 1 + idx - np.array([index_map.S(n, r - 1) for r in rows.tolist()], np.int64)
    np.testing.assert_array_equal(got, oracle.pairs(v.symbols, v.offsets, _pm1(), -1, rows, cols))
    for r0 in (0, 24950):
        b0, b1 = index_map.S(n, r0 - 1), index_map.S(n, r0 + 99)
        np.testing.assert_array_equal(out[b0:b1].cpu().numpy().astype(np.int32),
                                      oracle.triangle(v.symbols, v.offsets, _pm1(), -1, b0, b1),
                                      err_msg=f"rows {r0}..{r0 + 99}")


def test_batched_full_config_sampled_pairs():
    """The eight batched vocabularies (1k..100k words, int16 triangles, 22 GB of
    output) in one graph-replayed persistent run with the autotuner's setting:
    sampled pairs of every triangle against the oracle."""
    nw = _nw()
    _report("full size: batched config, 8 vocabularies")
    vocabs, S = synth.batched_configs()
    sc = nw.Scoring(64, submat=S, gap=-2)
    dvs = [nw.Vocab(v.symbols, v.offsets, sc) for v in vocabs]
    b = nw.Batch(dvs, torch.int16, class_width=1, wg_per_cu=8, pairs_per_item=16, use_graph=True)
    b.run()
    b.run()
    torch.cuda.synchronize()
    sim = oracle.sim_matrix(64, submat=S)
    rng = np.random.default_rng(8)
    for v, dv, o in zip(vocabs, dvs, b.outs):
        E = dv.num_pairs
        idx = np.unique(np.concatenate([rng.integers(0, E, 6000), np.arange(0, 20), np.arange(E - 20, E)]))
        got = o[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.int32)
        pi, pj = _pairs_of(v.n, idx)
        np.testing.assert_array_equal(got, oracle.pairs(v.symbols, v.offsets, sim, -2, pi, pj),
                                      err_msg=f"vocabulary of {v.n} words")
    b.close()


def test_served_queries_full_dictionary(paper):
    """The server on the 600,000-word dictionary (k = 16, 256 per batch, four
    slots), an open-loop burst at 20,000 q/s: every query's list equals the
    oracle's."""
    nw = _nw()
    _report("full size: served queries, 600k dictionary")
    v, dv = paper
    srv = nw.Server(dv, k=16, max_batch=256, num_slots=4)
    q = synth.query_words(160, seed=71)
    arr = synth.poisson_arrivals(20000.0, q.n, seed=72)
    s, i, lat = srv.replay(q.symbols, q.offsets, arr)
    srv.close()
    assert (lat > 0).all()
    ws, wi = oracle.query(v.symbols, v.offsets, _pm1(), -1, q.symbols, q.offsets, 16)
    np.testing.assert_array_equal(i, wi)
    np.testing.assert_array_equal(s.astype(np.int32), ws)
