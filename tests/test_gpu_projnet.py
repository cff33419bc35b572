"""The library's projectors against the definition of the explicit projector network T_P (SI B).

tn_read_projectors exports every P_L and P_R a run applied, with the bond they act on;
paper_2206_07044_amd.projector_network inserts them into the input network.  Contracted exactly
on the host (greedy pairwise order, not the tree's), T_P must give the run's own compressed
ln|Z| (float64 runs: to 1e-10 relative) on every compression path: the LDS core (D <= 64),
block Jacobi (both sides taller than 64 < D <= 256), the Gram-Lanczos core (D = 256), block
Krylov (D = 729 with an explicit side), Golub-Kahan-Lanczos (both sides taller than D = 300),
late compression, the tree gauge, a random-graph Agglom tree.
"""
import numpy as np
import pytest

import paper_2206_07044_amd as tn
from _exact_greedy import greedy_exact
from paper_2206_07044_amd._capi import TN_ESTATE, TNError
from tninputs import dimer_tensors, ising_tensors, lattice, normal_tensors, random_regular3
from tninputs.models import uniform_tensors
from tninputs.trees import agglom_tree, sweep_tree

pytestmark = pytest.mark.gpu


def _ctx(g, T):
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    c = tn.Context(0)
    c.tn_load_graph(g.n, eu, ev, ed, off, np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T]))
    return c


def _cases():
    g = lattice((6, 6))
    yield "ising-6x6-chi4", g, ising_tensors(g, 0.44), sweep_tree((6, 6)), 4, {}
    g = lattice((4, 4, 4))
    yield "normal-4x4x4-chi16-D256", g, normal_tensors(g, 0.1, seed=12), sweep_tree((4, 4, 4)), 16, {}
    g = lattice((3, 3, 3))
    yield "urand-3x3x3-chi2-late", g, uniform_tensors(g, -0.5, seed=3), sweep_tree((3, 3, 3)), 2, {"late": True}
    g = lattice((4, 4), dim=3)
    yield "normal-4x4-D3-chi3-gauge1", g, normal_tensors(g, 0.2, seed=4), sweep_tree((4, 4)), 3, {"gauge_r": 1}
    rr = random_regular3(20, seed=1)
    yield "dimer-rrg20-chi2", rr, dimer_tensors(rr), agglom_tree(rr, 2, seed=0), 2, {}
    g = lattice((3, 3, 4), dim=3)
    yield "normal-3x3x4-D3-chi27", g, normal_tensors(g, 0.2, seed=5), sweep_tree((3, 3, 4)), 27, {}
    from test_gpu_lanczos_degenerate import degenerate_network
    g, T, pairs, _ = degenerate_network(300, 600, 640, 0, "middle")
    yield "gkl-D300-chi6", g, T, pairs, 6, {}


CASES = list(_cases())


@pytest.mark.parametrize("name,g,T,pairs,chi,kw", CASES, ids=[c[0] for c in CASES])
def test_projector_network_of_the_gpu_run(name, g, T, pairs, chi, kw):
    pi, pj = [a for a, _ in pairs], [b for _, b in pairs]
    c = _ctx(g, T)
    try:
        c.tn_set_tree(pi, pj, chi, keep_intermediates=True, **kw)
        c.tn_contract_compressed()
        sign, lnz = c.tn_result()
        n_comp = len(c.tn_compress_stats()[0])
        n_p, edges_p, tens_p = tn.projector_network(c, g.n, g.edges, T, pi, pj, chi, late=kw.get("late", False))
        d256 = max(c.tn_read_projectors(k, values=False)["D"] for k in range(n_comp))
    finally:
        c.close()
    assert n_comp > 0 and n_p == g.n + 2 * n_comp
    sign_p, lnz_p = greedy_exact(n_p, edges_p, tens_p)
    print(f"{name}: {n_comp} compressions (largest bond {d256}), GPU ln|Z| {lnz!r}, T_P exact {lnz_p!r}", flush=True)
    assert sign_p == sign
    assert abs(lnz_p - lnz) <= 1e-10 * max(1.0, abs(lnz))


def test_read_projectors_needs_kept_buffers():
    g = lattice((4, 4))
    T = ising_tensors(g, 0.44)
    pairs = sweep_tree((4, 4))
    c = _ctx(g, T)
    try:
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], 2)
        bond = c.tn_read_projectors(0, values=False)   # the bond needs only the plan
        assert bond["D"] >= 2 and bond["chi"] == 2 and len(bond["edges"]) >= 1
        c.tn_contract_compressed()
        with pytest.raises(TNError) as e:
            c.tn_read_projectors(0)
        assert e.value.status == TN_ESTATE
    finally:
        c.close()


def test_frozen_projector_gradient():
    """d ln|Z| / d T_v with the run's projectors held fixed (frozen_projector_grad: the exact
    gradient of T_P through the library's reverse pass) against central differences of T_P's
    exact host contraction, the projectors kept, and Euler's identity <T_v, g_v> = 1 per input
    tensor (T_P is multilinear in the inputs)."""
    from tninputs import Graph
    from tninputs.trees import greedy_tree
    g = lattice((4, 4))
    T = ising_tensors(g, 0.44)
    pairs = sweep_tree((4, 4))
    pi, pj = [a for a, _ in pairs], [b for _, b in pairs]
    c = _ctx(g, T)
    try:
        c.tn_set_tree(pi, pj, 2, keep_intermediates=True)
        c.tn_contract_compressed()
        n_p, edges_p, _ = tn.projector_network(c, g.n, g.edges, T, pi, pj, 2)
        tree_p = greedy_tree(Graph(n_p, edges_p), 2 ** 30, seed=0)
        grads = tn.frozen_projector_grad(c, g.n, g.edges, T, pi, pj, 2, tree_p)
        euler = [float(np.sum(T[v] * grads[v])) for v in range(g.n)]
        print(f"Euler identity per tensor: max |<T, g> - 1| = {max(abs(e - 1.0) for e in euler):.2e}", flush=True)
        assert max(abs(e - 1.0) for e in euler) <= 1e-10
        rng = np.random.default_rng(7)
        h = 1e-6
        worst = 0.0
        for _ in range(6):
            v = int(rng.integers(g.n))
            idx = tuple(int(rng.integers(d)) for d in T[v].shape)
            vals = []
            for sgn in (1.0, -1.0):
                Tm = [t.copy() for t in T]
                Tm[v][idx] += sgn * h
                n2, e2, t2 = tn.projector_network(c, g.n, g.edges, Tm, pi, pj, 2)
                vals.append(greedy_exact(n2, e2, t2)[1])
            fd = (vals[0] - vals[1]) / (2 * h)
            worst = max(worst, abs(fd - grads[v][idx]))
        print(f"central differences of T_P: max |fd - g| = {worst:.2e}", flush=True)
        assert worst <= 1e-6
    finally:
        c.close()
