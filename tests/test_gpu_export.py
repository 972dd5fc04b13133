"""GPU parity of the streamed triangle export against the CPU oracle: the
chunks arrive in index order, cover the range exactly once, and hold the
oracle's scores; a callback can stop the export.  Every case prints its name
before the GPU work."""
import numpy as np
import pytest

import oracle
import synth
from oracle import index_map

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PM1 = dict(match=1, mismatch=-1, gap=-1)


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _vocab(v, submat=None, **kw):
    import paper_2509_01654_amd as nw
    return nw.Vocab(v.symbols, v.offsets, nw.Scoring(v.alphabet, submat=submat, **kw))


def _collect(dv, idx_begin, idx_end, chunk, dtype):
    got = np.zeros(idx_end - idx_begin, dtype=np.int32)
    seen = []

    def fn(b0, scores):
        seen.append((b0, len(scores)))
        got[b0 - idx_begin:b0 - idx_begin + len(scores)] = scores
        return False

    dv.export_triangle(fn, dtype=dtype, chunk_pairs=chunk, idx_begin=idx_begin, idx_end=idx_end)
    return got, seen


def _check_chunks(seen, idx_begin, idx_end, chunk):
    pos = idx_begin
    for b0, cnt in seen:
        assert b0 == pos and 0 < cnt <= chunk
        pos += cnt
    assert pos == idx_end
    assert len(seen) == -(-(idx_end - idx_begin) // chunk)


@pytest.mark.parametrize("dtype,chunk", [("int8", 300_001), ("int16", 1 << 18), ("int8", 1 << 30)])
def test_small_config_export(dtype, chunk):
    """2,000 words: every pair through ragged chunks equals the oracle's triangle."""
    _report(f"export small config {dtype} chunk={chunk}")
    v = synth.plain_config("small")
    dv = _vocab(v, **PM1)
    got, seen = _collect(dv, 0, dv.num_pairs, chunk, getattr(torch, dtype))
    _check_chunks(seen, 0, dv.num_pairs, chunk)
    np.testing.assert_array_equal(got, oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1))


def test_sub_range_and_single_pair_chunks():
    _report("export sub-range + one-pair chunks")
    v = synth.plain_config("small")
    dv = _vocab(v, **PM1)
    sim = oracle.sim_matrix(40, 1, -1)
    b0, b1 = 12_345, 1_500_000
    got, seen = _collect(dv, b0, b1, 99_999, torch.int16)
    _check_chunks(seen, b0, b1, 99_999)
    np.testing.assert_array_equal(got, oracle.triangle(v.symbols, v.offsets, sim, -1, b0, b1))
    t = synth.zipf_vocab(20, seed=31)
    dt = _vocab(t, **PM1)
    got, seen = _collect(dt, 0, dt.num_pairs, 1, torch.int8)
    _check_chunks(seen, 0, dt.num_pairs, 1)
    np.testing.assert_array_equal(got, oracle.triangle(t.symbols, t.offsets, sim, -1))
    # an empty range calls nothing
    got, seen = _collect(dt, 7, 7, 5, torch.int8)
    assert seen == []


def test_stop_and_exception():
    import paper_2509_01654_amd as nw
    _report("export stop + exception")
    v = synth.plain_config("small")
    dv = _vocab(v, **PM1)
    calls = []

    def stop_at_third(b0, scores):
        calls.append(b0)
        return len(calls) == 3

    with pytest.raises(nw.NwError) as e:
        dv.export_triangle(stop_at_third, chunk_pairs=100_000)
    assert e.value.code == nw.NW_ESTOPPED and len(calls) == 3

    def boom(b0, scores):
        raise ValueError("consumer failed")

    with pytest.raises(ValueError):
        dv.export_triangle(boom, chunk_pairs=100_000)
    # the dictionary still works afterwards
    got, _ = _collect(dv, 0, 1000, 256, torch.int8)
    np.testing.assert_array_equal(got, oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, 0,
                                                       1000))


def test_long_words_export():
    _report("export long words")
    v = synth.uniform_vocab(300, seed=93, alphabet=64, min_len=1, max_len=200)
    S = synth.random_submat(64, seed=4)
    dv = _vocab(v, submat=S, gap=-2)
    got, seen = _collect(dv, 0, dv.num_pairs, 7_777, torch.int16)
    _check_chunks(seen, 0, dv.num_pairs, 7_777)
    np.testing.assert_array_equal(got, oracle.triangle(v.symbols, v.offsets, oracle.sim_matrix(64, submat=S), -2))


def test_full_size_paper_workload_sampled():
    """600,000 words, the whole 1.8e11-byte int8 triangle through 2 x 1 GiB
    buffers: chunk order, sampled scores against the oracle, row boundaries."""
    _report("export 600k paper workload")
    v = synth.plain_config("paper")
    dv = _vocab(v, **PM1)
    n, E = v.n, dv.num_pairs
    rng = np.random.default_rng(11)
    chunk = 1 << 30
    samples = []
    starts = []

    def fn(b0, scores):
        starts.append((b0, len(scores)))
        off = rng.integers(0, len(scores), size=8)
        samples.extend(zip((b0 + off).tolist(), scores[off].tolist()))
        samples.append((b0, int(scores[0])))
        samples.append((b0 + len(scores) - 1, int(scores[-1])))
        return False

    dv.export_triangle(fn, dtype=torch.int8, chunk_pairs=chunk)
    _check_chunks(starts, 0, E, chunk)
    idx = np.array([s[0] for s in samples], np.int64)
    val = np.array([s[1] for s in samples], np.int32)
    pij = [index_map.pair_of_index(n, int(i)) for i in idx]
    pi = np.array([p[0] for p in pij], np.int64)
    pj = np.array([p[1] for p in pij], np.int64)
    want = oracle.pairs(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, pi, pj)
    np.testing.assert_array_equal(val, want)
