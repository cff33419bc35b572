"""Tensor values placed on a graph (SI section F of arXiv:2206.07044).

Every tensor is a dense float64 ``numpy`` array whose axes are the vertex's
incident edges in ascending edge id.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from .graphs import Graph

_H = np.array([[1.0, 1.0], [1.0, -1.0]])


def ising_bond_factors(beta: float, J: float):
    """Split exp(beta*J*s*s') into W_lo @ W_hi (SI F.1, the matrix W).

    Index 0 is spin +1 and index 1 is spin -1.  With c = cosh(beta J) and
    s = sinh(beta J), W_lo = H diag(sqrt c, sqrt|s|) H / sqrt 2 goes on the
    lower vertex id and W_hi = H diag(sqrt c, sign(s) sqrt|s|) H / sqrt 2 on the
    higher one.  For J > 0 both equal the paper's symmetric W; for J < 0 the
    sign of sinh goes to the higher-id side so the product is still the
    Boltzmann bond matrix.
    """
    c = np.cosh(beta * J)
    s = np.sinh(beta * J)
    w_lo = _H @ np.diag([np.sqrt(c), np.sqrt(abs(s))]) @ _H / np.sqrt(2.0)
    w_hi = _H @ np.diag([np.sqrt(c), np.sign(s) * np.sqrt(abs(s))]) @ _H / np.sqrt(2.0)
    return w_lo, w_hi


def ising_tensors(g: Graph, beta: float, J: Optional[Sequence[float]] = None) -> List[np.ndarray]:
    """T^[v]_{e...} = sum_s prod_{e at v} W^{(e)}_{s, e} (SI F.1).

    ``J`` gives one coupling per edge (default all +1).  All edges must have
    dimension 2.
    """
    if J is None:
        J = np.ones(g.n_edges)
    J = np.asarray(J, dtype=np.float64)
    inc = g.incident()
    facs = [ising_bond_factors(beta, float(J[e])) for e in range(g.n_edges)]
    out = []
    for v in range(g.n):
        mats = []
        for e in inc[v]:
            u, w, d = g.edges[e]
            if d != 2:
                raise ValueError("Ising edges have dimension 2")
            mats.append(facs[e][0] if v == u else facs[e][1])
        t = np.zeros((2,) * len(mats))
        for s in range(2):
            term = np.array(1.0)
            for m in mats:
                term = np.multiply.outer(term, m[s])
            t = t + term
        out.append(t)
    return out


def dimer_tensors(g: Graph) -> List[np.ndarray]:
    """T = 1 iff exactly one incident leg is 1 (SI F.3, dimer covers)."""
    inc = g.incident()
    out = []
    for v in range(g.n):
        k = len(inc[v])
        t = np.zeros((2,) * k)
        for a in range(k):
            idx = [0] * k
            idx[a] = 1
            t[tuple(idx)] = 1.0
        out.append(t)
    return out


def normal_tensors(g: Graph, mu: float, seed: int) -> List[np.ndarray]:
    """Entries i.i.d. Normal(mu, 1) from default_rng(seed), vertices in order."""
    rng = np.random.default_rng(seed)
    inc = g.incident()
    return [rng.normal(mu, 1.0, size=tuple(g.edges[e][2] for e in inc[v])) for v in range(g.n)]


def uniform_tensors(g: Graph, lam: float, seed: int) -> List[np.ndarray]:
    """URand model: entries i.i.d. Uniform[lam, 1] (main text II.B, SI F.2)."""
    rng = np.random.default_rng(seed)
    inc = g.incident()
    return [rng.uniform(lam, 1.0, size=tuple(g.edges[e][2] for e in inc[v])) for v in range(g.n)]
