"""Seeded synthetic inputs for compressed contraction-tree execution.

This package produces the *inputs* of the method of Gray & Chan,
"Hyper-optimized approximate contraction of tensor networks with arbitrary
geometry" (arXiv:2206.07044): tensor-network graphs, the tensors placed on
them (Ising, dimer, random models; SI section F) and fixed ordered
contraction trees (Greedy / Span / Agglom families, main text section II.G and SI
section C).  It holds none of the approximate-contraction arithmetic: both
the CPU oracle and the GPU library consume what it writes, and neither
imports the other.
"""
from .graphs import lattice, random_regular3, diamond, pyrochlore, Graph
from .models import ising_tensors, ising_bond_factors, dimer_tensors, normal_tensors, uniform_tensors
from .trees import greedy_tree, span_tree, agglom_tree, sweep_tree, simulate_tree, TreeStats
from .instance import Instance, save_instance, load_instance
from . import configs

__all__ = [
    "lattice", "random_regular3", "diamond", "pyrochlore", "Graph",
    "ising_tensors", "ising_bond_factors", "dimer_tensors", "normal_tensors", "uniform_tensors",
    "greedy_tree", "span_tree", "agglom_tree", "sweep_tree", "simulate_tree", "TreeStats",
    "Instance", "save_instance", "load_instance", "configs",
]
