"""Pins of the oracle's reference gradient (oracle/grad.py) against what does
not depend on it: central finite differences of the oracle's forward pass,
the Euler identity of a degree-1 homogeneous function, and, in the exact
regime, brute-force spin correlations (d ln Z / d J_e = beta <s_u s_v>).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from oracle.grad import ising_coupling_grad, lnz_and_grad
from tninputs import Graph, ising_tensors, lattice, normal_tensors, random_regular3
from tninputs.trees import sweep_tree


def _fd_directional(g, T, pairs, chi, dT, h):
    """Central difference of the oracle's ln|Z| along dT."""
    plus = [t + h * d for t, d in zip(T, dT)]
    minus = [t - h * d for t, d in zip(T, dT)]
    fp = oracle.contract_compressed(g.n, g.edges, plus, pairs, chi).ln_abs_z
    fm = oracle.contract_compressed(g.n, g.edges, minus, pairs, chi).ln_abs_z
    return (fp - fm) / (2.0 * h)


def _cases():
    g2 = lattice((4, 4))
    g3 = lattice((2, 2, 3))
    gd3 = lattice((3, 3), dim=3)
    rr = random_regular3(12, seed=5)
    multi = Graph(4, [(0, 1, 2), (0, 1, 3), (1, 2, 2), (2, 3, 2), (0, 3, 3), (1, 3, 2)])
    yield "ising-4x4-chi2", g2, ising_tensors(g2, 0.44), sweep_tree((4, 4)), 2
    yield "ising-4x4-chi3", g2, ising_tensors(g2, 0.44), sweep_tree((4, 4)), 3
    Jpm = np.where(np.random.default_rng(3).random(g3.n_edges) < 0.5, -1.0, 1.0)
    yield "pmJ-2x2x3-chi3", g3, ising_tensors(g3, 0.5, Jpm), sweep_tree((2, 2, 3)), 3
    yield "normal-3x3-D3-chi2", gd3, normal_tensors(gd3, 0.2, seed=1), sweep_tree((3, 3)), 2
    yield "normal-3x3-D3-chi4", gd3, normal_tensors(gd3, 0.0, seed=2), sweep_tree((3, 3)), 4
    pairs_rr = [(0, 1), (12, 2), (13, 3), (14, 4), (15, 5), (16, 6), (17, 7), (18, 8), (19, 9), (20, 10), (21, 11)]
    yield "normal-rrg12-chi3", rr, normal_tensors(rr, 0.1, seed=4), pairs_rr, 3
    yield "multi-edge-chi2", multi, normal_tensors(multi, 0.3, seed=6), [(0, 1), (2, 3), (4, 5)], 2


CASES = list(_cases())


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES, ids=[c[0] for c in CASES])
def test_gradient_matches_central_differences(name, g, T, pairs, chi):
    res = lnz_and_grad(g.n, g.edges, T, pairs, chi)
    ref = oracle.contract_compressed(g.n, g.edges, T, pairs, chi)
    assert res.ln_abs_z == pytest.approx(ref.ln_abs_z, rel=1e-13)
    assert res.sign == ref.sign
    rng = np.random.default_rng(11)
    for _ in range(2):
        dT = [rng.normal(size=t.shape) * np.max(np.abs(t)) for t in T]
        want = _fd_directional(g, T, pairs, chi, dT, 1e-5)
        got = sum(float(np.sum(gr * d)) for gr, d in zip(res.grads, dT))
        assert got == pytest.approx(want, rel=2e-6, abs=1e-8)


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES, ids=[c[0] for c in CASES])
def test_euler_identity(name, g, T, pairs, chi):
    # ln|Z| is degree-1 homogeneous in every input tensor, for any chi
    res = lnz_and_grad(g.n, g.edges, T, pairs, chi)
    for t, gr in zip(T, res.grads):
        assert float(np.sum(t * gr)) == pytest.approx(1.0, abs=1e-11)


# chi = 4096: no compression at all; the others compress rank-deficient cores
# (Ising copy-tensor structure) without truncating them, so ln Z is still exact
@pytest.mark.parametrize("shape,beta,seed,chi", [((3, 3), 0.44, None, 4096), ((2, 2, 2), 0.3, 1, 4096),
                                                 ((3, 4), 0.6, 2, 4096), ((3, 3), 0.44, None, 2),
                                                 ((3, 4), 0.6, 3, 2), ((4, 4), 0.44, 4, 4), ((2, 2, 3), 0.3, 5, 8)])
def test_exact_regime_matches_spin_correlations(shape, beta, seed, chi):
    g = lattice(shape)
    J = None if seed is None else np.where(np.random.default_rng(seed).random(g.n_edges) < 0.5, -1.0, 1.0)
    T = ising_tensors(g, beta, J)
    res = lnz_and_grad(g.n, g.edges, T, sweep_tree(shape), chi)
    assert res.ln_abs_z == pytest.approx(exact.ising_brute_force(g.n, g.edges, beta, J), rel=1e-13)
    dJ = ising_coupling_grad(g.n, g.edges, beta, np.ones(g.n_edges) if J is None else J, res.grads)
    want = beta * exact.ising_correlations_brute(g.n, g.edges, beta, J)
    np.testing.assert_allclose(dJ, want, rtol=1e-10, atol=1e-12)


def test_coupling_gradient_matches_finite_differences_truncated():
    shape, beta, chi = (4, 4), 0.5, 2
    g = lattice(shape)
    J = np.where(np.random.default_rng(7).random(g.n_edges) < 0.5, -1.0, 1.0)
    pairs = sweep_tree(shape)
    res = lnz_and_grad(g.n, g.edges, ising_tensors(g, beta, J), pairs, chi)
    dJ = ising_coupling_grad(g.n, g.edges, beta, J, res.grads)
    h = 1e-5
    for e in (0, 5, 11, g.n_edges - 1):
        Jp, Jm = J.copy(), J.copy()
        Jp[e] += h
        Jm[e] -= h
        fp = oracle.contract_compressed(g.n, g.edges, ising_tensors(g, beta, Jp), pairs, chi).ln_abs_z
        fm = oracle.contract_compressed(g.n, g.edges, ising_tensors(g, beta, Jm), pairs, chi).ln_abs_z
        assert dJ[e] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-9)


def test_ring_closed_form_derivative():
    # single cycle: ln Z = ln(prod 2cosh + prod 2sinh); derivative in closed form
    n, beta = 6, 0.7
    J = np.array([1.0, -1.0, 0.5, 2.0, -0.3, 1.2])
    g = Graph(n, sorted([(min(i, (i + 1) % n), max(i, (i + 1) % n), 2) for i in range(n)]))
    Jg = np.array([J[[i for i in range(n) if (min(i, (i + 1) % n), max(i, (i + 1) % n)) == (u, v)][0]]
                   for (u, v, _) in g.edges])
    T = ising_tensors(g, beta, Jg)
    pairs = [(0, 1), (6, 2), (7, 3), (8, 4), (9, 5)]
    res = lnz_and_grad(g.n, g.edges, T, pairs, 2)      # chi = 2: exact for a ring
    dJ = ising_coupling_grad(g.n, g.edges, beta, Jg, res.grads)
    c, s = np.cosh(beta * Jg), np.sinh(beta * Jg)
    pc, ps = np.prod(2 * c), np.prod(2 * s)
    want = beta * (pc * np.tanh(beta * Jg) + ps / np.tanh(beta * Jg)) / (pc + ps)
    np.testing.assert_allclose(dJ, want, rtol=1e-11)


def _probe_with_spectrum(sig, chi, seed):
    """One compression (tninputs.probes.bond_probe) of K = A_mat B_mat with singular values sig."""
    from tninputs.probes import bond_probe
    rng = np.random.default_rng(seed)
    D = len(sig)
    qa, _ = np.linalg.qr(rng.normal(size=(9, D)))
    qb, _ = np.linalg.qr(rng.normal(size=(9, D)))
    mix = np.linalg.qr(rng.normal(size=(D, D)))[0]          # A_mat and B_mat individually unstructured
    a_mat = qa @ np.diag(sig) @ mix
    b_mat = mix.T @ qb.T
    caps = [rng.normal(size=3) for _ in range(4)]
    return bond_probe(a_mat, b_mat, [D], (3, 3), (3, 3), caps), chi


@pytest.mark.parametrize("sig", [[3.0, 2.0, 2.0, 1.0, 0.5],          # exactly equal kept pair
                                 [3.0, 2.0, 2.0 - 1e-9, 1.0, 0.5],   # kept pair 1e-9 apart
                                 [2.0, 2.0, 2.0, 1.0, 0.5]])         # three equal kept values
def test_kept_degenerate_pairs_match_central_differences(sig):
    # the compression is smooth in K while the kept/discarded gap is open, however close the
    # kept values are: the gradient has a finite limit at an exact kept-kept degeneracy
    (g, T, pairs), chi = _probe_with_spectrum(np.array(sig), 3, seed=2)
    res = lnz_and_grad(g.n, g.edges, T, pairs, chi)
    rng = np.random.default_rng(5)
    for _ in range(3):
        dT = [rng.normal(size=t.shape) * np.max(np.abs(t)) for t in T]
        want = _fd_directional(g, T, pairs, chi, dT, 1e-6)
        got = sum(float(np.sum(gr * d)) for gr, d in zip(res.grads, dT))
        assert got == pytest.approx(want, rel=1e-6, abs=1e-8)


LATE_CASES = [c for c in CASES if c[0] in ("ising-4x4-chi2", "pmJ-2x2x3-chi3", "normal-3x3-D3-chi2", "normal-rrg12-chi3")]


@pytest.mark.parametrize("name,g,T,pairs,chi", LATE_CASES, ids=[c[0] for c in LATE_CASES])
def test_late_compression_gradient_matches_central_differences(name, g, T, pairs, chi):
    res = lnz_and_grad(g.n, g.edges, T, pairs, chi, compress_late=True)
    ref = oracle.contract_compressed(g.n, g.edges, T, pairs, chi, compress_late=True)
    assert res.ln_abs_z == pytest.approx(ref.ln_abs_z, rel=1e-13)
    assert any(o.kind == "compress" for o in ref.ops)
    rng = np.random.default_rng(12)
    for _ in range(2):
        dT = [rng.normal(size=t.shape) * np.max(np.abs(t)) for t in T]
        plus = [t + 1e-5 * d for t, d in zip(T, dT)]
        minus = [t - 1e-5 * d for t, d in zip(T, dT)]
        fp = oracle.contract_compressed(g.n, g.edges, plus, pairs, chi, compress_late=True).ln_abs_z
        fm = oracle.contract_compressed(g.n, g.edges, minus, pairs, chi, compress_late=True).ln_abs_z
        got = sum(float(np.sum(gr * d)) for gr, d in zip(res.grads, dT))
        assert got == pytest.approx((fp - fm) / 2e-5, rel=2e-6, abs=1e-8)
    for t, gr in zip(T, res.grads):
        assert float(np.sum(t * gr)) == pytest.approx(1.0, abs=1e-11)
