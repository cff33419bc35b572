"""Graph generators: open-boundary square/cubic, diamond and pyrochlore lattices and random
3-regular graphs.

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


def _cells(shape: Sequence[int]):
    L1, L2, L3 = (int(x) for x in shape)
    for k in range(L3):
        for j in range(L2):
            for i in range(L1):
                yield i, j, k


def diamond(shape: Sequence[int], dim: int = 2) -> Graph:
    """Open-boundary diamond lattice of L1 x L2 x L3 primitive fcc cells, two sites per cell
    (the "6x6x6(x2)" geometry of section IV.C has 432 sites).

    With fcc primitive vectors a1, a2, a3, the A site of cell R is joined to the B sites of cells
    R, R - a1, R - a2 and R - a3 (four bonds per site in the bulk).  Site ids: 2*c for A and
    2*c + 1 for B, c = i + L1*(j + L2*k).
    """
    L1, L2, L3 = (int(x) for x in shape)
    cid = lambda i, j, k: i + L1 * (j + L2 * k)
    raw = []
    for i, j, k in _cells(shape):
        a = 2 * cid(i, j, k)
        for di, dj, dk in ((0, 0, 0), (-1, 0, 0), (0, -1, 0), (0, 0, -1)):
            x, y, z = i + di, j + dj, k + dk
            if 0 <= x < L1 and 0 <= y < L2 and 0 <= z < L3:
                raw.append((a, 2 * cid(x, y, z) + 1))
    return _canon(2 * L1 * L2 * L3, raw, dim)


def pyrochlore(shape: Sequence[int], dim: int = 2) -> Graph:
    """Open-boundary pyrochlore lattice (corner-sharing tetrahedra) of L1 x L2 x L3 primitive
    fcc cells, four sites per cell.

    Sites s0..s3 of cell R form an "up" tetrahedron (all six pairs joined); the "down"
    tetrahedron joins s0(R), s1(R + a1), s2(R + a2) and s3(R + a3), the members that exist inside
    the open boundary.  Six bonds per site in the bulk.  Site ids: 4*c + s.
    """
    L1, L2, L3 = (int(x) for x in shape)
    cid = lambda i, j, k: i + L1 * (j + L2 * k)
    raw = []
    for i, j, k in _cells(shape):
        base = 4 * cid(i, j, k)
        for s in range(4):
            for t in range(s + 1, 4):
                raw.append((base + s, base + t))
        down = [base]
        for s, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1)), start=1):
            x, y, z = i + di, j + dj, k + dk
            if x < L1 and y < L2 and z < L3:
                down.append(4 * cid(x, y, z) + s)
        for a in range(len(down)):
            for b in range(a + 1, len(down)):
                raw.append((down[a], down[b]))
    return _canon(4 * L1 * L2 * L3, raw, dim)
