"""Graph generators: open-boundary square/cubic lattices and random 3-regular graphs.

A graph is ``n`` vertices and a list of edges ``(u, v, dim)`` with ``u < v``,
sorted lexicographically; the position of an edge in that list is its edge id.
The tensor on vertex ``v`` has one leg per incident edge, in ascending edge id
(the main text, section I, places one tensor per vertex and one index per edge).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


@dataclass
class Graph:
    n: int
    edges: List[Tuple[int, int, int]]  # (u, v, dim), u < v, sorted

    @property
    def n_edges(self) -> int:
        return len(self.edges)

    def incident(self) -> List[List[int]]:
        """Edge ids incident to each vertex, ascending (= the tensor's leg order)."""
        inc: List[List[int]] = [[] for _ in range(self.n)]
        for e, (u, v, _) in enumerate(self.edges):
            inc[u].append(e)
            inc[v].append(e)
        return inc

    def neighbors(self) -> List[List[int]]:
        nb: List[set] = [set() for _ in range(self.n)]
        for u, v, _ in self.edges:
            nb[u].add(v)
            nb[v].add(u)
        return [sorted(s) for s in nb]

    def arrays(self):
        e = np.asarray(self.edges, dtype=np.int64).reshape(-1, 3)
        return (e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int32))


def _canon(n: int, raw: Sequence[Tuple[int, int]], dim: int) -> Graph:
    edges = sorted({(min(u, v), max(u, v)) for u, v in raw})
    if len(edges) != len(raw):
        raise ValueError("duplicate edges")
    return Graph(n, [(u, v, dim) for u, v in edges])


def lattice(shape: Sequence[int], dim: int = 2) -> Graph:
    """Open-boundary hypercubic lattice.

    Vertex numbering is v = x + Lx*(y + Ly*z); nearest neighbours along every
    axis are joined by one edge of dimension ``dim``.
    """
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[:a])) for a in range(len(shape))]
    raw = []
    for v in range(n):
        rem = v
        coord = []
        for s in shape:
            coord.append(rem % s)
            rem //= s
        for a, s in enumerate(shape):
            if coord[a] + 1 < s:
                raw.append((v, v + strides[a]))
    return _canon(n, raw, dim)


def random_regular3(n: int, seed: int, dim: int = 2, max_tries: int = 100000) -> Graph:
    """Random simple 3-regular graph from the pairing (configuration) model.

    Three stubs per vertex are shuffled with ``numpy.random.default_rng(seed)``
    and paired consecutively; a pairing with a self-loop or a repeated edge is
    rejected and redrawn from the same generator.
    """
    if n % 2 or n < 4:
        raise ValueError("a 3-regular graph needs an even n >= 4")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n), 3)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        canon = np.sort(pairs, axis=1)
        key = canon[:, 0].astype(np.int64) * n + canon[:, 1]
        if np.unique(key).size != key.size:
            continue
        return _canon(n, [tuple(p) for p in canon.tolist()], dim)
    raise RuntimeError("could not draw a simple 3-regular graph")
