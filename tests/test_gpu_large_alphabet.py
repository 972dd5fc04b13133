"""Every call on a 255-symbol alphabet with a wide similarity matrix: the
profiles (256 rows) are the largest the register-row kernels stage in LDS,
and the top-k histogram (961 bins) fits in LDS beside them for short row
lengths but not for the longest, so one call exercises both histogram paths.
Everything against the oracle, bit-exact."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A = 255


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def big():
    import paper_2509_01654_amd as nw
    v = synth.uniform_vocab(1500, seed=95, alphabet=A, min_len=1, max_len=48)
    S = synth.random_submat(A, seed=96, lo=-10, hi=10, diag=10)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(A, submat=S, gap=-1))
    sim = oracle.sim_matrix(A, submat=S)
    return v, S, dv, sim, oracle.triangle(v.symbols, v.offsets, sim, -1)


def test_triangle(big):
    _report("large alphabet: triangle")
    v, S, dv, sim, tri = big
    got = dv.all_pairs_scores(dtype=torch.int16)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy().astype(np.int32), tri)
    diag = dv.all_pairs_scores_diag(dtype=torch.int16)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(diag.cpu().numpy().astype(np.int32), tri)


def test_topk_and_histogram(big):
    _report("large alphabet: top-8 + histogram")
    v, S, dv, sim, tri = big
    lo, hi = dv.bounds
    assert hi - lo + 1 > 900   # wide enough that the longest rows keep their bins outside LDS
    s, i, h = dv.all_pairs_topk(8)
    torch.cuda.synchronize()
    ws, wi, wh = oracle.topk_rows(v.symbols, v.offsets, sim, -1, 8, hist_range=(lo, hi))
    np.testing.assert_array_equal(i.cpu().numpy(), wi)
    np.testing.assert_array_equal(s.cpu().numpy().astype(np.int32), ws)
    np.testing.assert_array_equal(h.cpu().numpy().astype(np.uint64), wh)
    np.testing.assert_array_equal(wh, np.bincount(tri - lo, minlength=hi - lo + 1).astype(np.uint64))


def test_queries(big):
    _report("large alphabet: queries")
    v, S, dv, sim, tri = big
    q = synth.uniform_vocab(40, seed=97, alphabet=A, min_len=1, max_len=48)
    s, i = dv.query(q.symbols, q.offsets, 6)
    torch.cuda.synchronize()
    ws, wi = oracle.query(v.symbols, v.offsets, sim, -1, q.symbols, q.offsets, 6)
    np.testing.assert_array_equal(i.cpu().numpy(), wi)
    np.testing.assert_array_equal(s.cpu().numpy().astype(np.int32), ws)


def test_edges(big):
    _report("large alphabet: edges")
    v, S, dv, sim, tri = big
    i, j, s, count = dv.all_pairs_edges(200, 400, normalised=False)
    torch.cuda.synchronize()
    wi, wj, ws = oracle.edges(v.symbols, v.offsets, sim, -1, 200, 400, False)
    assert count == len(wi) > 100
    key = i.cpu().numpy()[:count].astype(np.int64) * v.n + j.cpu().numpy()[:count]
    order = np.argsort(key)
    np.testing.assert_array_equal(key[order], np.asarray(wi, np.int64) * v.n + np.asarray(wj, np.int64))
    np.testing.assert_array_equal(s.cpu().numpy()[:count][order].astype(np.int32), ws)


def test_batched(big):
    import paper_2509_01654_amd as nw
    _report("large alphabet: batched")
    v, S, dv, sim, tri = big
    b = nw.Batch([dv], torch.int16, class_width=8, wg_per_cu=4, pairs_per_item=16, use_graph=False)
    out = b.run()[0]
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy()[:tri.shape[0]].astype(np.int32), tri)
    b.close()
