"""nw_query_noalloc (the query entry point that allocates nothing, its
workspace in the library's fixed device scratch) against nw_query on the same
dictionary and queries: bit-exact, on two calls in a row, the second with a
smaller batch, plus the host-side refusals."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _noalloc(lib):
    fn = lib.nw_query_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return fn


def _call(nw, dv, q, k, stream=None):
    lib = nw.load_library()
    sc = torch.full((max(q.n, 1), k), 7, dtype=torch.int16, device=dv.device)
    ix = torch.full((max(q.n, 1), k), 7, dtype=torch.int32, device=dv.device)
    rc = _noalloc(lib)(dv._h, q.symbols.ctypes.data, q.offsets.ctypes.data, q.n, k, ctypes.c_void_p(sc.data_ptr()),
                       ctypes.c_void_p(ix.data_ptr()), nw._stream_handle(stream))
    if rc != nw.NW_OK:
        raise nw.NwError(rc, lib.nw_last_error().decode())
    torch.cuda.synchronize()
    return sc[:q.n].cpu().numpy(), ix[:q.n].cpu().numpy()


@pytest.fixture(scope="module")
def dictionary():
    import paper_2509_01654_amd as nw
    v = synth.zipf_vocab(20000, seed=70, mean_len=8.0, max_len=32)
    return nw, nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))


def test_noalloc_equals_query_two_calls(dictionary):
    nw, dv = dictionary
    k = 16
    # first call: 200 queries of mixed lengths, including empty and 32-symbol words
    _report("no-alloc query: 200 queries, k = 16")
    rng = np.random.default_rng(71)
    words = [synth.query_words(198, seed=72).word(t) for t in range(198)] + [np.zeros(0, np.uint8),
                                                                               rng.integers(0, 40, 32)]
    q1 = synth.vocab_from_words(words, 40)
    s1, i1 = _call(nw, dv, q1, k)
    w1 = dv.query(q1.symbols, q1.offsets, k)
    np.testing.assert_array_equal(i1, w1[1].cpu().numpy())
    np.testing.assert_array_equal(s1, w1[0].cpu().numpy())
    # second call, smaller: 37 queries (the scratch keeps the first call's contents)
    _report("no-alloc query: 37 queries, k = 16, after the larger call")
    q2 = synth.query_words(37, seed=73)
    s2, i2 = _call(nw, dv, q2, k)
    w2 = dv.query(q2.symbols, q2.offsets, k)
    np.testing.assert_array_equal(i2, w2[1].cpu().numpy())
    np.testing.assert_array_equal(s2, w2[0].cpu().numpy())
    # one query at the largest k (the most column splits per query)
    _report("no-alloc query: 1 query, k = 64")
    q3 = synth.query_words(1, seed=74)
    s3, i3 = _call(nw, dv, q3, 64)
    w3 = dv.query(q3.symbols, q3.offsets, 64)
    np.testing.assert_array_equal(i3, w3[1].cpu().numpy())
    np.testing.assert_array_equal(s3, w3[0].cpu().numpy())


def test_noalloc_refuses_on_the_host(dictionary):
    nw, dv = dictionary
    _report("no-alloc query: host-side refusals")
    with pytest.raises(nw.NwError) as e:
        _call(nw, dv, synth.query_words(257, seed=75), 8)
    assert e.value.code == nw.NW_EINVAL and "at most 256" in str(e.value)
    with pytest.raises(nw.NwError) as e:
        _call(nw, dv, synth.query_words(3, seed=76), 65)
    assert e.value.code == nw.NW_EINVAL
    bad = synth.vocab_from_words([[1, 2], [40]], 40)
    with pytest.raises(nw.NwError) as e:
        _call(nw, dv, bad, 8)
    assert e.value.code == nw.NW_EINVAL
