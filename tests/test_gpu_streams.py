"""Stream semantics of the calls whose launches are spread over library
streams: work the caller enqueues after a call on the same stream sees the
call's complete output, with no device synchronisation in between; and a
captured graph of such a call replays to the same output."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def vocab():
    import paper_2509_01654_amd as nw
    v = synth.zipf_vocab(3000, seed=61, mean_len=8.0, max_len=32)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    tri = oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1)
    return v, dv, tri


def test_triangle_then_same_stream_reduction(vocab):
    _report("streams: triangle then reduction on the caller's stream")
    v, dv, tri = vocab
    s = torch.cuda.Stream()
    want = int(tri.astype(np.int64).sum())
    sums = []
    with torch.cuda.stream(s):
        out = torch.empty(dv.num_pairs, dtype=torch.int16, device="cuda")
        for _ in range(4):
            out.fill_(0)
            dv.all_pairs_scores(dtype=torch.int16, out=out, stream=s)
            sums.append(out.to(torch.int64).sum())
    s.synchronize()
    assert [int(x) for x in sums] == [want] * 4


def test_topk_then_same_stream_reduction(vocab):
    _report("streams: top-k then reduction on the caller's stream")
    v, dv, tri = vocab
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        sc, ix, h = dv.all_pairs_topk(8, stream=s)
        total = h.sum()
        first = sc[:, 0].to(torch.int64).sum()
    s.synchronize()
    assert int(total) == v.n * (v.n - 1) // 2
    ws, wi, _ = oracle.topk_rows(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, 8)
    assert int(first) == int(ws[:, 0].astype(np.int64).sum())


def test_triangle_graph_capture_replays(vocab):
    _report("streams: captured triangle call, several replays")
    v, dv, tri = vocab
    out = torch.zeros(dv.num_pairs, dtype=torch.int16, device="cuda")
    dv.all_pairs_scores(dtype=torch.int16, out=out)   # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=s):
        dv.all_pairs_scores(dtype=torch.int16, out=out, stream=s)
    for _ in range(3):
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().astype(np.int32), tri)
