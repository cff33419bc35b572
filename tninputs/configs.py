"""Named workloads: the seeded instances the benchmark and the tests run.

Each function returns ``(graph, tensors, pairs)``: the tensor network (one
tensor per vertex, axes in ascending edge id) and the ordered contraction
tree.  Sizes are the ones the workloads are measured at; every random choice
comes from ``numpy.random.default_rng`` with the seed given.

* ``cubic_ising``      3D Ising, J = 1 (SI F.1), Span-family sweep tree.
* ``spin_glass``       3D +-J spin glass (SI F.1): couplings +-1 with equal probability.
* ``square_ising``     2D Ising on L x L (SI F.1) with the seed-0 Greedy tree.
* ``dimer_rrg``        dimer covers of a random 3-regular graph (section IV.B, SI F.3),
                       Agglom-family tree.
* ``normal_rrg``       Normal(mu, 1) tensors of bond dimension D on a random 3-regular graph
                       (section IV.C, SI F.2), Agglom-family tree.
* ``urand_lattice``    URand tensors, entries uniform in [lambda, 1] (section III), on the
                       square, cubic, diamond or pyrochlore lattice.
* ``pyrochlore_ising`` ferromagnetic Ising model on the pyrochlore lattice (section IV.A).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .graphs import Graph, diamond, lattice, pyrochlore, random_regular3
from .models import dimer_tensors, ising_tensors, normal_tensors, uniform_tensors
from .trees import agglom_tree, greedy_tree, span_tree, sweep_tree

Workload = Tuple[Graph, List[np.ndarray], List[Tuple[int, int]]]


def pm_couplings(n_edges: int, seed: int = 0) -> np.ndarray:
    """+-1 couplings with equal probability: J_e = -1 where default_rng(seed).random() < 1/2."""
    return np.where(np.random.default_rng(seed).random(n_edges) < 0.5, -1.0, 1.0)


def cubic_ising(L: int = 12, beta: float = 0.22) -> Workload:
    g = lattice((L, L, L))
    return g, ising_tensors(g, beta), sweep_tree((L, L, L))


def spin_glass(L: int = 16, beta: float = 0.5, seed: int = 0) -> Workload:
    g = lattice((L, L, L))
    return g, ising_tensors(g, beta, pm_couplings(g.n_edges, seed)), sweep_tree((L, L, L))


def square_ising(L: int = 8, beta: float = 0.44, tree_chi: int = 256) -> Workload:
    g = lattice((L, L))
    return g, ising_tensors(g, beta), greedy_tree(g, tree_chi, 0)


def dimer_rrg(n: int, chi: int, seed: int = 0, k: int = 4, tree_seed: int = 0) -> Workload:
    """Dimer tensors (one nonzero per unit-weight configuration) on random_regular3(n, seed)."""
    g = random_regular3(n, seed)
    return g, dimer_tensors(g), agglom_tree(g, chi, k=k, seed=tree_seed)


def normal_rrg(n: int, mu: float, chi: int, seed: int = 0, tensor_seed: int = 0, D: int = 3, k: int = 4,
               tree_seed: int = 0) -> Workload:
    g = random_regular3(n, seed, dim=D)
    return g, normal_tensors(g, mu, tensor_seed), agglom_tree(g, chi, k=k, seed=tree_seed)


def urand_lattice(kind: str, shape: Sequence[int], lam: float, chi: int, seed: int = 0, D: int = 2,
                  tree: str = "span") -> Workload:
    """URand tensors on ``kind`` in {'square', 'cubic', 'diamond', 'pyrochlore'}."""
    if kind in ("square", "cubic"):
        g = lattice(shape, dim=D)
    elif kind == "diamond":
        g = diamond(shape, dim=D)
    elif kind == "pyrochlore":
        g = pyrochlore(shape, dim=D)
    else:
        raise ValueError(f"unknown lattice {kind!r}")
    T = uniform_tensors(g, lam, seed)
    return g, T, lattice_tree(g, kind, shape, chi, tree)


def lattice_tree(g: Graph, kind: str, shape: Sequence[int], chi: int, tree: str = "span") -> List[Tuple[int, int]]:
    """'span': the axis sweep on square/cubic lattices, else span_tree(g, seed=0); 'span-corner':
    span_tree grown from the least central vertex with distance-only scoring (no connectivity
    term, no noise), the boundary-like sweep that keeps diamond and pyrochlore intermediates
    small; 'greedy' and 'agglom': those families with seed 0."""
    if tree == "span":
        pairs = sweep_tree(shape) if kind in ("square", "cubic") else span_tree(g, seed=0)
    elif tree == "span-corner":
        pairs = span_tree(g, seed=0, start="min", temperature=0.0, w_connectivity=0.0)
    elif tree == "greedy":
        pairs = greedy_tree(g, chi, 0)
    else:
        pairs = agglom_tree(g, chi, seed=0)
    return pairs


def pyrochlore_ising(L: int, beta: float, chi: int) -> Workload:
    """Ferromagnetic Ising model (J = 1, spins along one common axis) on the L^3 x 4 pyrochlore
    lattice of section IV.A, on the 'span-corner' tree."""
    g = pyrochlore((L, L, L))
    return g, ising_tensors(g, beta), lattice_tree(g, "pyrochlore", (L, L, L), chi, "span-corner")
