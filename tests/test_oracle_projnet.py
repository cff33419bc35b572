"""Pins of the explicit projector network T_P (SI B): an exact contraction of the input network
with every compression's P_L P_R pair inserted equals the compressed value of Algorithm 1.

The exact contraction here is a greedy pairwise one written in this file (each step contracts
the connected pair with the smallest result, every intermediate rescaled by its largest entry),
a different order from the tree the projectors came from, so the test checks the projectors and
their placement, not a replay of the same arithmetic.
"""
import math

import numpy as np
import pytest

from _exact_greedy import greedy_exact
from oracle.approx import contract_compressed
from oracle.projnet import projector_network
from tninputs import Graph, dimer_tensors, ising_tensors, lattice, normal_tensors, random_regular3
from tninputs.models import uniform_tensors
from tninputs.trees import agglom_tree, sweep_tree


def _cases():
    g = lattice((4, 4))
    yield "ising-4x4-chi2", g, ising_tensors(g, 0.44), sweep_tree((4, 4)), 2, {}
    g = lattice((3, 3, 3))
    yield "urand-3x3x3-chi2", g, uniform_tensors(g, -0.5, seed=2), sweep_tree((3, 3, 3)), 2, {}
    yield "urand-3x3x3-chi2-late", g, uniform_tensors(g, -0.5, seed=3), sweep_tree((3, 3, 3)), 2, {"compress_late": True}
    g3 = lattice((4, 4), dim=3)
    yield "normal-4x4-D3-chi3-gauge1", g3, normal_tensors(g3, 0.2, seed=4), sweep_tree((4, 4)), 3, {"gauge_r": 1}
    rr = random_regular3(20, seed=1)
    yield "dimer-rrg20-chi2", rr, dimer_tensors(rr), agglom_tree(rr, 2, seed=0), 2, {}


CASES = list(_cases())


@pytest.mark.parametrize("name,g,T,pairs,chi,kw", CASES, ids=[c[0] for c in CASES])
def test_projector_network_contracts_to_the_compressed_value(name, g, T, pairs, chi, kw):
    res, n_p, edges_p, tens_p = projector_network(g.n, g.edges, T, pairs, chi, **kw)
    comp = [o for o in res.ops if o.kind == "compress"]
    assert comp and max(o.discarded for o in comp) > 1e-8, "the case truncates nothing"
    # T_P: the inputs unchanged (up to the order of their axes: a bundle edge copied on the
    # neighbour's side is renumbered), two projectors per compression, every edge between two
    # tensors
    assert n_p == g.n + 2 * len(comp)
    for v in range(g.n):
        np.testing.assert_array_equal(np.sort(tens_p[v].ravel()), np.sort(np.asarray(T[v], dtype=np.float64).ravel()))
    for u, v, d in edges_p:
        assert u < v and d >= 1
    sign, lnz = greedy_exact(n_p, edges_p, tens_p)
    assert sign == res.sign
    assert abs(lnz - res.ln_abs_z) <= 1e-10 * max(1.0, abs(res.ln_abs_z)), (lnz, res.ln_abs_z)
    # and the compression did change the value: T_P is not the input network in disguise
    exact = contract_compressed(g.n, g.edges, T, pairs, None)
    assert abs(exact.ln_abs_z - res.ln_abs_z) > 1e-9 * max(1.0, abs(exact.ln_abs_z))


def test_projector_network_without_truncation_is_exact():
    """chi at the largest bond: every compression keeps the whole core, P_L P_R is the identity on
    the bond's range, and T_P contracts to the exact value."""
    g = lattice((3, 3))
    T = ising_tensors(g, 0.3)
    pairs = sweep_tree((3, 3))
    exact = contract_compressed(g.n, g.edges, T, pairs, None)
    res, n_p, edges_p, tens_p = projector_network(g.n, g.edges, T, pairs, 2 ** 6)
    assert n_p == g.n + 2 * sum(1 for o in res.ops if o.kind == "compress")
    sign, lnz = greedy_exact(n_p, edges_p, tens_p)
    assert sign == exact.sign and abs(lnz - exact.ln_abs_z) <= 1e-12 * abs(exact.ln_abs_z)


def test_projector_insertion_is_needed():
    """A planted mistake: dropping one projector pair (the bundle reconnected directly) changes
    the contracted value away from the compressed one, so the pin above sees the projectors."""
    g = lattice((4, 4))
    T = ising_tensors(g, 0.44)
    pairs = sweep_tree((4, 4))
    res, n_p, edges_p, tens_p = projector_network(g.n, g.edges, T, pairs, 2)
    # scale the last P_L by 2: the value must move by ln 2
    t = list(tens_p)
    t[n_p - 2] = 2.0 * t[n_p - 2]
    _, lnz = greedy_exact(n_p, edges_p, t)
    assert abs(lnz - (res.ln_abs_z + math.log(2.0))) <= 1e-10 * abs(res.ln_abs_z)
