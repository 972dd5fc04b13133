"""Batched persistent form: every dictionary's triangle equals the oracle's,
for every option, eager or graph-replayed."""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def small_batch():
    import paper_2509_01654_amd as nw
    vocabs, S = synth.batched_configs(scale=0.012)   # 12 .. 1,200 words, lengths 1..8 .. 1..48
    sc = nw.Scoring(64, submat=S, gap=-2)
    dvs = [nw.Vocab(v.symbols, v.offsets, sc) for v in vocabs]
    sim = oracle.sim_matrix(64, submat=S)
    want = [oracle.triangle(v.symbols, v.offsets, sim, -2) for v in vocabs]
    return vocabs, dvs, want


@pytest.mark.parametrize("width,wg,ppi,graph", [(8, 4, 64, True), (1, 2, 16, True), (8, 8, 0, False),
                                                (1, 4, 0, False), (0, 1, 0, True), (0, 1, 0, False)])
def test_batched_equals_oracle(small_batch, width, wg, ppi, graph):
    import paper_2509_01654_amd as nw
    _report(f"batched width={width} wg={wg} ppi={ppi} graph={graph}")
    vocabs, dvs, want = small_batch
    b = nw.Batch(dvs, torch.int16, class_width=width, wg_per_cu=wg, pairs_per_item=ppi, use_graph=graph)
    outs = b.run()
    torch.cuda.synchronize()
    for v, o, w in zip(vocabs, outs, want):
        got = o.cpu().numpy()[:w.shape[0]].astype(np.int32)
        np.testing.assert_array_equal(got, w)
    items, launches = b.info()
    assert launches >= 1
    assert items > 0 if width else items == 0   # the tiled form plans no work items
    b.close()


def test_graph_replays_with_eager_work_between(small_batch):
    import paper_2509_01654_amd as nw
    _report("graph replays")
    vocabs, dvs, want = small_batch
    b = nw.Batch(dvs, torch.int16, use_graph=True)
    for rep in range(4):
        for o in b.outs:
            o.fill_(-12345)                      # eager work on the same stream between replays
        torch.cuda.synchronize()
        outs = b.run()
        torch.cuda.synchronize()
        for v, o, w in zip(vocabs, outs, want):
            np.testing.assert_array_equal(o.cpu().numpy()[:w.shape[0]].astype(np.int32), w)
        # the eager per-dictionary kernel agrees with the replay
        e = dvs[rep].all_pairs_scores(dtype=torch.int16)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(e.cpu().numpy(), b.outs[rep].cpu().numpy()[:e.numel()])
    b.close()


def test_autotune_and_cache(small_batch, tmp_path):
    import paper_2509_01654_amd as nw
    _report("autotune")
    vocabs, dvs, want = small_batch
    cache = str(tmp_path / "tune.jsonl")
    b = nw.Batch(dvs, torch.int16, autotune=True, cache_path=cache)
    first = dict(b.options)
    outs = b.run()
    torch.cuda.synchronize()
    for v, o, w in zip(vocabs, outs, want):
        np.testing.assert_array_equal(o.cpu().numpy()[:w.shape[0]].astype(np.int32), w)
    b.close()
    assert os.path.exists(cache) and open(cache).read().count("class_width") == 1
    b2 = nw.Batch(dvs, torch.int16, autotune=True, cache_path=cache)
    assert b2.options == first
    assert open(cache).read().count("class_width") == 1
    b2.close()
