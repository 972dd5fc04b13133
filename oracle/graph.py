"""Ego networks of the word graph (TEST INFRASTRUCTURE ONLY, like the rest of
this package).

Section 5 reads the word graph through ego networks: the words within a few
hops (depth 3 in its figures) of a chosen word, in a slice of edge weights.
An ego network is fixed by hop distances: breadth-first search from the seed
words over the undirected graph, stopped at the depth.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def adjacency(n: int, ei, ej):
    """Neighbour lists of the undirected graph with edges {ei[e], ej[e]} on n nodes."""
    adj = [[] for _ in range(n)]
    for a, b in zip(np.asarray(ei).tolist(), np.asarray(ej).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    return adj


def ego_network(n: int, ei, ej, seeds, depth: int) -> np.ndarray:
    """Hop distance from the nearest seed (0 for the seeds) for every node within
    `depth` hops, -1 for the others: breadth-first search, one level at a time."""
    adj = adjacency(n, ei, ej)
    dist = np.full(n, -1, dtype=np.int32)
    queue = deque()
    for s in np.asarray(seeds, dtype=np.int64).tolist():
        if dist[s] < 0:
            dist[s] = 0
            queue.append(s)
    while queue:
        v = queue.popleft()
        if dist[v] == depth:
            continue
        for u in adj[v]:
            if dist[u] < 0:
                dist[u] = dist[v] + 1
                queue.append(u)
    return dist
