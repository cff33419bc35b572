"""Exact references that pin the oracle — TEST INFRASTRUCTURE ONLY.

None of these uses tensor networks: they sum the physical model directly
(Ising partition function, SI Eq. (ising-partition-fn); dimer covers, SI F.3)
so that they are independent of both the oracle and the GPU library.
"""
from __future__ import annotations

import math
from functools import lru_cache
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


def _couplings(n_edges: int, J) -> np.ndarray:
    return np.ones(n_edges) if J is None else np.asarray(J, dtype=np.float64)


def ising_brute_force(n: int, edges: Sequence[Tuple[int, int, int]], beta: float, J=None) -> float:
    """ln Z with Z = sum over all 2^n spin states of prod_edges exp(beta J s_u s_v)."""
    if n > 22:
        raise ValueError("brute force is limited to 22 spins")
    J = _couplings(len(edges), J)
    states = np.arange(2 ** n, dtype=np.int64)
    spins = 1 - 2 * ((states[:, None] >> np.arange(n)) & 1)   # bit 0 -> +1
    energy = np.zeros(2 ** n)
    for e, (u, v, _) in enumerate(edges):
        energy += J[e] * spins[:, u] * spins[:, v]
    x = beta * energy
    mx = x.max()
    return float(mx + math.log(np.sum(np.exp(x - mx))))


def ising_transfer_matrix(shape: Sequence[int], beta: float, J=None,
                          edges: Optional[Sequence[Tuple[int, int, int]]] = None) -> float:
    """ln Z of the open-boundary lattice Ising model by a layer transfer matrix.

    Layers are slices along the last axis (vertex v = x + Lx*(y + ...)); the
    state of a layer is the tuple of its spins, so the cost is 4^(layer size)
    per layer.  ``edges``/``J`` give per-edge couplings (default all +1).
    """
    shape = tuple(int(s) for s in shape)
    layer = int(np.prod(shape[:-1]))
    nl = shape[-1]
    if layer > 12:
        raise ValueError("layer too large for a transfer matrix")
    if edges is None:
        from tninputs import lattice  # graph only, no tensor arithmetic
        edges = lattice(shape).edges
    J = _couplings(len(edges), J)
    S = 2 ** layer
    st = np.arange(S, dtype=np.int64)
    spins = 1 - 2 * ((st[:, None] >> np.arange(layer)) & 1)   # (S, layer)
    intra = [np.zeros(S) for _ in range(nl)]
    inter = [np.zeros((S, S)) for _ in range(nl - 1)]
    for e, (u, v, _) in enumerate(edges):
        lu, lv = u // layer, v // layer
        pu, pv = u % layer, v % layer
        if lu == lv:
            intra[lu] += J[e] * spins[:, pu] * spins[:, pv]
        else:
            assert lv == lu + 1
            inter[lu] += J[e] * np.outer(spins[:, pu], spins[:, pv])
    # log-domain forward recursion
    logv = beta * intra[0]
    for l in range(nl - 1):
        m = logv.max()
        w = np.exp(logv - m) @ np.exp(beta * inter[l])
        logv = m + np.log(w) + beta * intra[l + 1]
    m = logv.max()
    return float(m + math.log(np.sum(np.exp(logv - m))))


def ising_forest(n: int, edges: Sequence[Tuple[int, int, int]], beta: float, J=None) -> float:
    """Closed form for a graph without cycles: Z = 2^(#components) prod_e 2 cosh(beta J_e)."""
    J = _couplings(len(edges), J)
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v, _ in edges:
        ru, rv = find(u), find(v)
        if ru == rv:
            raise ValueError("graph has a cycle")
        parent[ru] = rv
    comps = len({find(x) for x in range(n)})
    return comps * math.log(2.0) + float(np.sum(np.log(2.0 * np.cosh(beta * J))))


def ising_ring(beta: float, J: Sequence[float]) -> float:
    """Closed form for a single cycle: Z = prod 2cosh(beta J) + prod 2sinh(beta J)."""
    J = np.asarray(J, dtype=np.float64)
    return math.log(np.prod(2 * np.cosh(beta * J)) + np.prod(2 * np.sinh(beta * J)))


def ising_correlations_brute(n: int, edges, beta: float, J=None) -> np.ndarray:
    """<s_u s_v> for every edge by brute force; d ln Z / d J_e = beta <s_u s_v>."""
    J = _couplings(len(edges), J)
    states = np.arange(2 ** n, dtype=np.int64)
    spins = 1 - 2 * ((states[:, None] >> np.arange(n)) & 1)
    energy = np.zeros(2 ** n)
    prods = []
    for e, (u, v, _) in enumerate(edges):
        p = spins[:, u] * spins[:, v]
        prods.append(p)
        energy += J[e] * p
    x = beta * energy
    w = np.exp(x - x.max())
    w /= w.sum()
    return np.array([float(np.sum(w * p)) for p in prods])


def perfect_matchings(n: int, edges: Sequence[Tuple[int, int, int]]) -> int:
    """Number of perfect matchings (dimer covers) by memoised search over vertex masks."""
    if n > 40:
        raise ValueError("too many vertices for the exact matching count")
    adj = [0] * n
    for u, v, _ in edges:
        adj[u] |= 1 << v
        adj[v] |= 1 << u
    full = (1 << n) - 1

    @lru_cache(maxsize=None)
    def count(mask: int) -> int:
        if mask == full:
            return 1
        free = ~mask & full
        v = (free & -free).bit_length() - 1
        cand = adj[v] & free
        tot = 0
        while cand:
            u = (cand & -cand).bit_length() - 1
            cand &= cand - 1
            tot += count(mask | (1 << v) | (1 << u))
        return tot

    return count(0)


def einsum_contract(n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray]) -> float:
    """Exact value of a small closed network via numpy.einsum (library routine)."""
    import string
    letters = string.ascii_letters
    if len(edges) > len(letters):
        raise ValueError("too many edges for einsum")
    inc: List[List[int]] = [[] for _ in range(n)]
    for e, (u, v, _) in enumerate(edges):
        inc[u].append(e)
        inc[v].append(e)
    spec = ",".join("".join(letters[e] for e in sorted(inc[v])) for v in range(n)) + "->"
    return float(np.einsum(spec, *tensors, optimize="greedy"))
