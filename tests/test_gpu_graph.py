"""GPU parity of the word-graph calls (compressed rows, ego networks) against
the CPU oracle.  Rows are compared as sorted neighbour multisets (their order
is free); distances element by element.  Every case prints its name first."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from oracle import graph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _nw():
    import paper_2509_01654_amd as nw
    return nw


def _report(name):
    print(f"[gpu case] {name}", flush=True)


def _edges_on_gpu(ei, ej):
    return (torch.from_numpy(np.ascontiguousarray(ei, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ej, dtype=np.int32)).cuda())


def _check_rows(n, ei, ej, row_ptr, adj):
    deg = np.bincount(np.concatenate([ei, ej]).astype(np.int64), minlength=n) if len(ei) else np.zeros(n, np.int64)
    rp = row_ptr.cpu().numpy()
    np.testing.assert_array_equal(rp, np.concatenate([[0], np.cumsum(deg)]))
    a = adj.cpu().numpy()
    ref = graph.adjacency(n, ei, ej)
    for v in range(n):
        assert sorted(a[rp[v]:rp[v + 1]].tolist()) == sorted(ref[v]), v


CASES = [(1, 0), (2, 1), (10, 30), (257, 400), (1000, 2500), (5000, 4000), (3000, 60000)]


@pytest.mark.parametrize("n,m", CASES)
def test_random_graphs(n, m):
    _report(f"graph random n={n} m={m}")
    nw = _nw()
    rng = np.random.default_rng(400 + n + m)
    ei = rng.integers(0, n, size=m)
    ej = rng.integers(0, n, size=m)          # self-loops and repeats included
    gi, gj = _edges_on_gpu(ei, ej)
    row_ptr, adj = nw.graph_csr(n, gi, gj)
    torch.cuda.synchronize()
    _check_rows(n, ei, ej, row_ptr, adj)
    for seeds, depth in (([0], 0), ([0], 1), ([n - 1, 0, n // 2], 3), ([n // 3] * 3, 6)):
        dist = nw.ego_network(row_ptr, adj, seeds, depth)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dist.cpu().numpy(), graph.ego_network(n, ei, ej, seeds, depth))


def test_many_seeds_and_empty_graph():
    _report("graph many seeds + empty graph")
    nw = _nw()
    rng = np.random.default_rng(77)
    n = 2000
    ei, ej = rng.integers(0, n, 3000), rng.integers(0, n, 3000)
    row_ptr, adj = nw.graph_csr(n, *_edges_on_gpu(ei, ej))
    seeds = rng.integers(0, n, size=300)     # several seeding launches
    dist = nw.ego_network(row_ptr, adj, seeds, 2)
    np.testing.assert_array_equal(dist.cpu().numpy(), graph.ego_network(n, ei, ej, seeds, 2))
    e0 = torch.empty(0, dtype=torch.int32, device="cuda")
    row_ptr, adj = nw.graph_csr(50, e0, e0)
    assert row_ptr.cpu().numpy().tolist() == [0] * 51
    dist = nw.ego_network(row_ptr, adj, [7], 3)
    np.testing.assert_array_equal(dist.cpu().numpy(), graph.ego_network(50, [], [], [7], 3))
    dist = nw.ego_network(row_ptr, adj, [], 3)
    assert (dist.cpu().numpy() == -1).all()


def test_word_graph_from_edge_slices():
    """Edges of the 2,000-word dictionary in the normalised slice [40, 100], then
    ego networks of depth 3 (the paper's depth) around a few words."""
    _report("graph from edge slice, small config")
    nw = _nw()
    v = synth.plain_config("small")
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    i, j, s, count = dv.all_pairs_edges(40, 100, True, 1)
    row_ptr, adj = nw.graph_csr(v.n, i, j)
    wi, wj, _ = oracle.edges(v.symbols, v.offsets, oracle.sim_matrix(40, 1, -1), -1, 40, 100, True, 1)
    assert count == len(wi)
    _check_rows(v.n, wi, wj, row_ptr, adj)
    for seeds in ([0], [5, 1999], list(range(0, 2000, 97))):
        dist = nw.ego_network(row_ptr, adj, seeds, 3)
        np.testing.assert_array_equal(dist.cpu().numpy(), graph.ego_network(v.n, wi, wj, seeds, 3))


def test_argument_errors():
    _report("graph argument errors")
    nw = _nw()
    lib = nw.load_library()
    n = 10
    for bad in ([0, 10], [-1, 3]):
        gi, gj = _edges_on_gpu(np.array([1, bad[0]]), np.array([2, bad[1]]))
        with pytest.raises(nw.NwError) as e:
            nw.graph_csr(n, gi, gj)
        assert e.value.code == nw.NW_EINVAL
    gi, gj = _edges_on_gpu(np.array([1]), np.array([2]))
    row_ptr, adj = nw.graph_csr(n, gi, gj)
    with pytest.raises(nw.NwError) as e:
        nw.ego_network(row_ptr, adj, [10], 1)
    assert e.value.code == nw.NW_EINVAL
    with pytest.raises(nw.NwError) as e:
        nw.ego_network(row_ptr, adj, [1], 1_000_001)
    assert e.value.code == nw.NW_EINVAL
    need = ctypes.c_uint64()
    assert lib.nw_graph_workspace_bytes(n, ctypes.byref(need)) == 0
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    rp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ad = torch.empty(2, dtype=torch.int32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert lib.nw_graph_csr(n, P(gi), P(gj), 1, P(rp), P(ad), P(ws), need.value - 1,
                            nw._stream_handle(None)) == nw.NW_ENOMEM


def test_full_size_ego_networks():
    """600,000 words: the normalised slice [60, 100] as a graph, ego networks of
    depth 3 around sampled words against breadth-first search on the CPU."""
    _report("graph 600k paper workload")
    nw = _nw()
    v = synth.plain_config("paper")
    dv = nw.Vocab(v.symbols, v.offsets, nw.Scoring(40, 1, -1, -1))
    i, j, s, count = dv.all_pairs_edges(60, 100, True, 1)
    row_ptr, adj = nw.graph_csr(v.n, i, j)
    ei, ej = i.cpu().numpy(), j.cpu().numpy()
    deg = np.bincount(np.concatenate([ei, ej]).astype(np.int64), minlength=v.n)
    np.testing.assert_array_equal(row_ptr.cpu().numpy(), np.concatenate([[0], np.cumsum(deg)]))
    rng = np.random.default_rng(12)
    hubs = np.argsort(deg)[-2:]              # the best-connected words and random ones
    for seeds in ([int(hubs[-1])], rng.integers(0, v.n, size=5).tolist(), [int(hubs[-2]), 17]):
        dist = nw.ego_network(row_ptr, adj, seeds, 3)
        np.testing.assert_array_equal(dist.cpu().numpy(), graph.ego_network(v.n, ei, ej, seeds, 3))
