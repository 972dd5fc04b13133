"""The continuous-batching query server: each result equals the query run alone
(and the oracle), whatever batch and slot it ran in."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


@pytest.fixture(scope="module")
def dictionary():
    import paper_2509_01654_amd as nw
    v = synth.zipf_vocab(20000, seed=60, mean_len=8.0, max_len=32)
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    return v, dv


def _alone(dv, q, k):
    """Each query through nw_query on its own."""
    s_all, i_all = [], []
    for t in range(q.n):
        w = q.word(t)
        s, i = dv.query(w, np.array([0, w.shape[0]], np.uint64), k)
        s_all.append(s.cpu().numpy()[0])
        i_all.append(i.cpu().numpy()[0])
    return np.array(s_all), np.array(i_all)


def test_replay_mix_equals_alone_and_oracle(dictionary):
    import paper_2509_01654_amd as nw
    _report("server replay 600 queries at 20k q/s")
    v, dv = dictionary
    q = synth.query_words(600, seed=61)
    k = 16
    arrivals = synth.poisson_arrivals(20000.0, q.n, seed=62)
    srv = nw.Server(dv, k=k, max_batch=64, num_slots=4)
    sc, ix, lat = srv.replay(q.symbols, q.offsets, arrivals)
    batches, queries = srv.stats()
    srv.close()
    assert queries == q.n and batches >= 1
    assert (lat > 0).all()
    s1, i1 = _alone(dv, q, k)
    np.testing.assert_array_equal(ix, i1)
    np.testing.assert_array_equal(sc, s1)
    sim = oracle.sim_matrix(40, 1, -1)
    sub = np.arange(0, q.n, 7)
    qs = q.subset(sub)
    ws, wi = oracle.query(v.symbols, v.offsets, sim, -1, qs.symbols, qs.offsets, k)
    np.testing.assert_array_equal(ix[sub], wi)
    np.testing.assert_array_equal(sc[sub].astype(np.int32), ws)


def test_submit_poll_burst_mixed_lengths(dictionary):
    import paper_2509_01654_amd as nw
    _report("server submit/poll burst")
    v, dv = dictionary
    rng = np.random.default_rng(63)
    words = [rng.integers(0, 40, size=int(rng.integers(0, 49))) for _ in range(300)] + [[], [5], [5] * 48]
    q = synth.vocab_from_words(words, 40)
    k = 8
    srv = nw.Server(dv, k=k, max_batch=32, num_slots=3)
    for t in range(q.n):
        srv.submit(q.word(t), tag=t)
    got = {}
    while len(got) < q.n:
        tags, sc, ix, lat = srv.poll(256, 100000)
        for t, s, i in zip(tags, sc, ix):
            got[int(t)] = (s.copy(), i.copy())
    srv.close()
    s1, i1 = _alone(dv, q, k)
    for t in range(q.n):
        np.testing.assert_array_equal(got[t][1], i1[t])
        np.testing.assert_array_equal(got[t][0], s1[t])


def test_server_rejects_bad_queries(dictionary):
    import paper_2509_01654_amd as nw
    _report("server argument errors")
    _, dv = dictionary
    srv = nw.Server(dv, k=4, max_batch=8, num_slots=1)
    with pytest.raises(nw.NwError):
        srv.submit(np.zeros(49, np.uint8), tag=0)
    with pytest.raises(nw.NwError):
        srv.submit(np.array([40], np.uint8), tag=1)
    srv.close()


def test_admission_by_memory_with_a_capped_pool(dictionary):
    """A pool that holds about one small batch at a time: batches wait or
    shrink for memory, never exceed the pool, and every result is still the
    query's result alone."""
    import paper_2509_01654_amd as nw
    _report("server with a capped workspace pool")
    v, dv = dictionary
    k = 16
    least = nw.Server.min_workspace_bytes(dv, k)
    pool = 3 * least
    srv = nw.Server(dv, k=k, max_batch=64, num_slots=4, ws_bytes=pool)
    q = synth.query_words(400, seed=64)
    for t in range(q.n):
        srv.submit(q.word(t), tag=t)
    got = {}
    while len(got) < q.n:
        tags, sc, ix, lat = srv.poll(256, 100000)
        for t, s, i in zip(tags, sc, ix):
            got[int(t)] = (s.copy(), i.copy())
    size, peak, waits = srv.memory_stats()
    batches, queries = srv.stats()
    srv.close()
    assert size <= pool and 0 < peak <= size
    assert waits >= 1 and queries == q.n and batches >= 2
    s1, i1 = _alone(dv, q, k)
    for t in range(q.n):
        np.testing.assert_array_equal(got[t][1], i1[t])
        np.testing.assert_array_equal(got[t][0], s1[t])
    with pytest.raises(nw.NwError) as e:
        nw.Server(dv, k=k, max_batch=8, num_slots=1, ws_bytes=least - 256)
    assert e.value.code == nw.NW_ENOMEM


def test_failed_launch_stops_admission_and_destroy_returns(dictionary):
    """A batch that fails on the host (injected before anything is enqueued):
    the server reports the error, drops what was queued, and closing it
    returns even though requests were still waiting."""
    import time
    import paper_2509_01654_amd as nw
    _report("server error path: injected host-side failure")
    _, dv = dictionary
    srv = nw.Server(dv, k=8, max_batch=4, num_slots=1)
    srv.inject_failure()
    q = synth.query_words(64, seed=65)
    for t in range(q.n):
        try:
            srv.submit(q.word(t), tag=t)
        except nw.NwError as e:
            assert e.code == nw.NW_EDEVICE
            break
    t0 = time.time()
    with pytest.raises(nw.NwError) as e:
        while time.time() - t0 < 30:
            srv.poll(64, 100000)
    assert e.value.code == nw.NW_EDEVICE and "injected" in str(e.value)
    t1 = time.time()
    srv.close()
    assert time.time() - t1 < 10
