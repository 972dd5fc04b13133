"""Graph capture at the boundary: the calls that wait for the device or use
host callbacks refuse a capturing stream with NW_EINVAL (nothing enqueued);
the capture-safe calls (the one-call batched triangles here) replay to the
oracle's output; the enqueue-only top-k and its finishing call give the
blocking call's result."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def small():
    import paper_2509_01654_amd as nw
    v = synth.zipf_vocab(3000, seed=81, mean_len=8.0, max_len=32)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    return nw, v, dv


def test_query_and_topk_refuse_a_capturing_stream(small):
    nw, v, dv = small
    _report("capture: nw_query and nw_all_pairs_topk refuse a capturing stream")
    q = synth.query_words(4, seed=82)
    ws = torch.empty(dv.query_workspace_bytes(q.n, 8), dtype=torch.uint8, device="cuda")
    out = (torch.empty((q.n, 8), dtype=torch.int16, device="cuda"), torch.empty((q.n, 8), dtype=torch.int32,
                                                                                device="cuda"))
    kws = torch.empty(dv.topk_workspace_bytes(8), dtype=torch.uint8, device="cuda")
    kout = (torch.empty((dv.n, 8), dtype=torch.int16, device="cuda"),
            torch.empty((dv.n, 8), dtype=torch.int32, device="cuda"),
            torch.empty(dv.bounds[1] - dv.bounds[0] + 1, dtype=torch.int64, device="cuda"))
    x = torch.zeros(16, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    codes = []
    with torch.cuda.graph(g, stream=s):
        x.add_(1.0)
        for call in (lambda: dv.query(q.symbols, q.offsets, 8, ws=ws, out=out, stream=s),
                     lambda: dv.all_pairs_topk(8, ws=kws, out=kout, stream=s),
                     lambda: dv.all_pairs_topk_async(8, kws, kout, stream=s)):
            try:
                call()
                codes.append(nw.NW_OK)
            except nw.NwError as e:
                codes.append(e.code)
                assert "captured" in str(e)
    assert codes == [nw.NW_EINVAL] * 3
    g.replay()
    torch.cuda.synchronize()
    assert float(x[0]) == 1.0
    # the same calls work once the capture is over
    sc, ix = dv.query(q.symbols, q.offsets, 8, ws=ws, out=out)
    torch.cuda.synchronize()
    ws_, wi = oracle.query(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, q.symbols, q.offsets, 8)
    np.testing.assert_array_equal(ix.cpu().numpy(), wi)


def test_batched_one_call_eager_and_captured():
    import paper_2509_01654_amd as nw
    vocabs, S = synth.batched_configs(scale=0.012)
    sc = nw.Scoring(64, submat=S, gap=-2)
    dvs = [nw.Vocab(v.symbols, v.offsets, sc) for v in vocabs]
    sim = oracle.sim_matrix(64, submat=S)
    want = [oracle.triangle(v.symbols, v.offsets, sim, -2) for v in vocabs]
    _report("nw_all_pairs_scores_batched eager")
    outs = nw.all_pairs_scores_batched(dvs, torch.int16)
    torch.cuda.synchronize()
    for o, w in zip(outs, want):
        np.testing.assert_array_equal(o.cpu().numpy()[:w.shape[0]].astype(np.int32), w)
    _report("nw_all_pairs_scores_batched captured, four replays")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        nw.all_pairs_scores_batched(dvs, torch.int16, outs=outs, stream=s)
    for _ in range(4):
        for o in outs:
            o.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            np.testing.assert_array_equal(o.cpu().numpy()[:w.shape[0]].astype(np.int32), w)


def test_topk_async_then_finish_equals_blocking(small):
    nw, v, dv = small
    _report("top-k enqueue-only form + finish")
    k = 16
    ws = torch.empty(dv.topk_workspace_bytes(k), dtype=torch.uint8, device="cuda")
    out = (torch.empty((dv.n, k), dtype=torch.int16, device="cuda"),
           torch.empty((dv.n, k), dtype=torch.int32, device="cuda"),
           torch.empty(dv.bounds[1] - dv.bounds[0] + 1, dtype=torch.int64, device="cuda"))
    with pytest.raises(nw.NwError) as e:
        dv.topk_finish(k, ws, out)
    assert e.value.code == nw.NW_EINVAL and "pending" in str(e.value)
    dv.all_pairs_topk_async(k, ws, out)
    dv.topk_finish(k, ws, out)
    torch.cuda.synchronize()
    a = [t.cpu().numpy().copy() for t in out]
    b = dv.all_pairs_topk(k)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y.cpu().numpy())
    lo, hi = dv.bounds
    ws_, wi, wh = oracle.topk_rows(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, k, hist_range=(lo, hi))
    np.testing.assert_array_equal(a[1], wi)
    np.testing.assert_array_equal(a[0].astype(np.int32), ws_)
    np.testing.assert_array_equal(a[2].astype(np.uint64), wh)
