"""Pins of the oracle's ego networks (hop distances by breadth-first search).

Reachability by powers of the adjacency matrix (a node is within d hops of a
seed exactly when (I + A)^d links them), SciPy's unweighted shortest paths,
and hand-made graphs fix the distances; planted mistakes must fail a pin.
CPU only.
"""
import numpy as np
import pytest

from oracle import graph


def _random_graph(rng, n, m, loops=True):
    ei = rng.integers(0, n, size=m)
    ej = rng.integers(0, n, size=m)
    if not loops:
        keep = ei != ej
        ei, ej = ei[keep], ej[keep]
    return ei.astype(np.int64), ej.astype(np.int64)


def _by_matrix_powers(n, ei, ej, seeds, depth):
    A = np.zeros((n, n), dtype=np.int64)
    A[ei, ej] = 1
    A[ej, ei] = 1
    step = ((A + np.eye(n, dtype=np.int64)) > 0).astype(np.int64)
    reach = np.zeros(n, dtype=bool)
    reach[np.asarray(seeds, dtype=np.int64)] = True
    dist = np.where(reach, 0, -1).astype(np.int32)
    for d in range(1, depth + 1):
        reach = (reach.astype(np.int64) @ step) > 0
        dist[(dist < 0) & reach] = d
    return dist


def test_hand_made_graphs():
    # a path 0-1-2-3-4-5, a triangle 6-7-8, an isolated node 9, a self-loop at 9
    ei = np.array([0, 1, 2, 3, 4, 6, 7, 8, 9])
    ej = np.array([1, 2, 3, 4, 5, 7, 8, 6, 9])
    assert graph.ego_network(10, ei, ej, [0], 3).tolist() == [0, 1, 2, 3, -1, -1, -1, -1, -1, -1]
    assert graph.ego_network(10, ei, ej, [5], 0).tolist() == [-1] * 5 + [0] + [-1] * 4
    assert graph.ego_network(10, ei, ej, [2, 7], 1).tolist() == [-1, 1, 0, 1, -1, -1, 1, 0, 1, -1]
    assert graph.ego_network(10, ei, ej, [9, 9], 5).tolist() == [-1] * 9 + [0]
    # edges count in both directions: seeding the far end of the path reaches back
    assert graph.ego_network(10, ei, ej, [4], 2).tolist()[2:7] == [2, 1, 0, 1, -1]


@pytest.mark.parametrize("seed", range(6))
def test_distances_equal_matrix_powers(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(5, 40))
    ei, ej = _random_graph(rng, n, int(rng.integers(0, 3 * n)))
    seeds = rng.integers(0, n, size=int(rng.integers(1, 4)))
    for depth in (0, 1, 2, 3, 5):
        np.testing.assert_array_equal(graph.ego_network(n, ei, ej, seeds, depth),
                                      _by_matrix_powers(n, ei, ej, seeds, depth))


def test_distances_equal_scipy_shortest_paths():
    sp = pytest.importorskip("scipy.sparse")
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    rng = np.random.default_rng(9)
    n = 400
    ei, ej = _random_graph(rng, n, 500, loops=False)
    A = sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(n, n)).tocsr()
    seeds = [3, 250]
    D = csgraph.shortest_path(A, directed=False, unweighted=True, indices=seeds).min(axis=0)
    for depth in (1, 3, 6):
        want = np.where(D <= depth, D, -1).astype(np.int32)
        np.testing.assert_array_equal(graph.ego_network(n, ei, ej, seeds, depth), want)


_REAL = graph.adjacency


def _directed_only(n, ei, ej):
    adj = [[] for _ in range(n)]
    for a, b in zip(np.asarray(ei).tolist(), np.asarray(ej).tolist()):
        adj[a].append(b)
    return adj


def _drops_first_edge(n, ei, ej):
    return _REAL(n, np.asarray(ei)[1:], np.asarray(ej)[1:])


def _ego_depth_plus_one(n, ei, ej, seeds, depth, _f=graph.ego_network):
    return _f(n, ei, ej, seeds, depth + 1)


def _ego_seeds_at_one(n, ei, ej, seeds, depth, _f=graph.ego_network):
    d = _f(n, ei, ej, seeds, depth)
    return np.where(d >= 0, d + 1, -1).astype(np.int32)


@pytest.mark.parametrize("name", ["directed_only", "drops_first_edge", "depth_plus_one", "seeds_at_one"])
def test_pins_catch_mutants(name, monkeypatch):
    if name == "directed_only":
        monkeypatch.setattr(graph, "adjacency", _directed_only)
    elif name == "drops_first_edge":
        monkeypatch.setattr(graph, "adjacency", _drops_first_edge)
    elif name == "depth_plus_one":
        monkeypatch.setattr(graph, "ego_network", _ego_depth_plus_one)
    else:
        monkeypatch.setattr(graph, "ego_network", _ego_seeds_at_one)
    caught = 0
    for t in (test_hand_made_graphs, lambda: [test_distances_equal_matrix_powers(s) for s in range(6)],
              test_distances_equal_scipy_shortest_paths):
        try:
            t()
        except AssertionError:
            caught += 1
    assert caught, f"no pin caught mutant {name}"
