"""Host-side checks of the new input generators: the diamond and pyrochlore lattices, the
Agglom-family tree builder and the named workloads (no GPU, no oracle arithmetic beyond a
brute-force check on a tiny diamond)."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from tninputs import agglom_tree, configs, diamond, ising_tensors, pyrochlore, random_regular3, simulate_tree


def _degrees(g):
    deg = np.zeros(g.n, dtype=int)
    for u, v, _ in g.edges:
        deg[u] += 1
        deg[v] += 1
    return deg


def test_diamond_is_bipartite_four_regular_in_the_bulk():
    g = diamond((4, 4, 4))
    assert g.n == 128
    deg = _degrees(g)
    assert deg.max() == 4
    # an A site (even id) away from the lower faces has all four bonds
    assert deg[2 * (1 + 4 * (1 + 4 * 1))] == 4
    assert all((u % 2) != (v % 2) for u, v, _ in g.edges)          # A-B bonds only
    # bonds = 4 per A site minus the missing ones on the open faces
    assert g.n_edges == sum(1 + (i > 0) + (j > 0) + (k > 0) for i in range(4) for j in range(4) for k in range(4))


def test_pyrochlore_corner_sharing_tetrahedra():
    g = pyrochlore((3, 3, 3))
    assert g.n == 108
    deg = _degrees(g)
    assert deg.max() == 6
    nb = g.neighbors()
    # the bulk site s0 of cell (1,1,1) has 6 bonds, each in a triangle of its tetrahedron, and
    # its two tetrahedra share only that site
    v = 4 * (1 + 3 * (1 + 3 * 1))
    assert deg[v] == 6
    for u in nb[v]:
        assert len(set(nb[u]) & set(nb[v])) == 2
    up = {v + 1, v + 2, v + 3}
    assert up <= set(nb[v]) and len(set(nb[v]) - up) == 3


def test_ising_on_tiny_diamond_matches_brute_force():
    g = diamond((2, 2, 1))
    T = ising_tensors(g, 0.4)
    pairs = agglom_tree(g, 64, k=4, seed=0)
    r = oracle.contract_compressed(g.n, g.edges, T, pairs, 64)
    assert r.ln_abs_z == pytest.approx(exact.ising_brute_force(g.n, g.edges, 0.4, None), rel=1e-13)


@pytest.mark.parametrize("n,chi,k", [(40, 4, 4), (64, 2, 8), (100, 8, 16)])
def test_agglom_tree_is_a_valid_ordered_tree(n, chi, k):
    g = random_regular3(n, 1)
    pairs = agglom_tree(g, chi, k=k, seed=3)
    assert len(pairs) == g.n - 1
    live = set(range(g.n))
    for t, (a, b) in enumerate(pairs):
        assert a in live and b in live and a != b
        live -= {a, b}
        live.add(g.n + t)
    assert len(live) == 1
    assert pairs == agglom_tree(g, chi, k=k, seed=3)              # seeded: reproducible
    assert simulate_tree(g, pairs, chi).n_compress > 0            # merged parts share composite bonds


def test_agglom_beats_single_region_growth_on_random_graphs():
    # section IV.B: partition-based trees suit random graphs; a tree that grows one region keeps
    # every boundary bond separate and never compresses
    from tninputs import greedy_tree
    g = random_regular3(200, 0)
    a = simulate_tree(g, agglom_tree(g, 4, k=4, seed=0), 4)
    gr = simulate_tree(g, greedy_tree(g, 4, 0, temperature=0.0), 4)
    assert a.largest_elems < gr.largest_elems
    assert a.n_compress >= 50


def test_named_workloads_shapes():
    g, T, p = configs.spin_glass(4)
    assert g.n == 64 and len(p) == 63 and len(T) == 64
    J = configs.pm_couplings(g.n_edges, 0)
    assert set(np.unique(J)) <= {-1.0, 1.0}
    g, T, p = configs.dimer_rrg(40, 4)
    assert all(t.sum() == 3 for t in T)                            # one dimer per vertex: three patterns
    g, T, p = configs.normal_rrg(20, 0.2, 2)
    assert all(t.shape == (3, 3, 3) for t in T)
    for kind, shape in (("diamond", (2, 2, 2)), ("pyrochlore", (2, 2, 1)), ("square", (4, 4)), ("cubic", (2, 2, 3))):
        g, T, p = configs.urand_lattice(kind, shape, -0.5, 8)
        assert len(p) == g.n - 1 and all(np.all(t >= -0.5) and np.all(t <= 1.0) for t in T)
