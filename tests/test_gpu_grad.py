"""GPU reverse pass (tn_grad) against the oracle's reference gradient.

Every case runs the same seeded inputs and tree through the C ABI and through
oracle.grad; the FP64 form must match element by element, the Euler identity
<T_v, d ln|Z|/d T_v> = 1 must hold for every input tensor, and in the exact
regime the coupling gradient must equal beta <s_u s_v> by brute force.
"""
import math

import numpy as np
import pytest

import paper_2206_07044_amd as tn
from oracle import exact
from oracle.grad import ising_coupling_grad, lnz_and_grad
from tninputs import Graph, ising_tensors, lattice, normal_tensors, random_regular3
from tninputs.trees import sweep_tree

pytestmark = pytest.mark.gpu

# |g_gpu - g_oracle| <= GRAD_RTOL * max|g_oracle| (FP64 end to end; the adjoint divides by
# singular values and gaps, so it is allowed a few digits more than ln Z's 1e-10)
GRAD_RTOL = 1e-9
FP32_GRAD_RTOL = 2e-3


def flat(g, T):
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    return eu, ev, ed, off, np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T])


def gpu_grad(g, T, pairs, chi, precision="fp64"):
    eu, ev, ed, off, data = flat(g, T)
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision, grad=True)
        c.tn_contract_compressed()
        sign, lnz = c.tn_result()
        gflat = c.tn_grad()
        disc, tie, sw = c.tn_compress_stats()
    finally:
        c.close()
    grads = [gflat[off[v]:off[v + 1]].reshape(T[v].shape) for v in range(g.n)]
    return sign, lnz, grads, tie


def _cases():
    g2 = lattice((4, 4))
    g3 = lattice((2, 2, 3))
    gd3 = lattice((3, 3), dim=3)
    rr = random_regular3(12, seed=5)
    multi = Graph(4, [(0, 1, 2), (0, 1, 3), (1, 2, 2), (2, 3, 2), (0, 3, 3), (1, 3, 2)])
    g8 = lattice((8, 8))
    g4 = lattice((4, 4, 4))
    yield "ising-4x4-chi2", g2, ising_tensors(g2, 0.44), sweep_tree((4, 4)), 2
    yield "ising-4x4-chi3", g2, ising_tensors(g2, 0.44), sweep_tree((4, 4)), 3
    Jpm = np.where(np.random.default_rng(3).random(g3.n_edges) < 0.5, -1.0, 1.0)
    yield "pmJ-2x2x3-chi3", g3, ising_tensors(g3, 0.5, Jpm), sweep_tree((2, 2, 3)), 3
    yield "normal-3x3-D3-chi2", gd3, normal_tensors(gd3, 0.2, seed=1), sweep_tree((3, 3)), 2
    yield "normal-3x3-D3-chi4", gd3, normal_tensors(gd3, 0.0, seed=2), sweep_tree((3, 3)), 4
    pairs_rr = [(0, 1)] + [(12 + t, t + 2) for t in range(10)]
    yield "normal-rrg12-chi3", rr, normal_tensors(rr, 0.1, seed=4), pairs_rr, 3
    yield "multi-edge-chi2", multi, normal_tensors(multi, 0.3, seed=6), [(0, 1), (2, 3), (4, 5)], 2
    yield "ising-8x8-chi8", g8, ising_tensors(g8, 0.44), sweep_tree((8, 8)), 8
    J4 = np.where(np.random.default_rng(9).random(g4.n_edges) < 0.5, -1.0, 1.0)
    yield "pmJ-4x4x4-chi4", g4, ising_tensors(g4, 0.5, J4), sweep_tree((4, 4, 4)), 4
    yield "normal-4x4x4-chi6", g4, normal_tensors(g4, 0.3, seed=3), sweep_tree((4, 4, 4)), 6
    g6 = lattice((6, 6, 6))      # long reductions: split-K contraction adjoints
    J6 = np.where(np.random.default_rng(0).random(g6.n_edges) < 0.5, -1.0, 1.0)
    yield "pmJ-6x6x6-chi8", g6, ising_tensors(g6, 0.5, J6), sweep_tree((6, 6, 6)), 8
    # bonds of D = chi^2 > 64: the global core path (blocked pivoted Cholesky, block Jacobi over
    # 16-column blocks, MFMA projectors); D = 100 and 144 leave partial blocks, 256 fills 16
    yield "normal-4x4x4-chi10-D100", g4, normal_tensors(g4, 0.3, seed=11), sweep_tree((4, 4, 4)), 10
    yield "pmJ-4x4x4-chi12-D144", g4, ising_tensors(g4, 0.5, J4), sweep_tree((4, 4, 4)), 12
    yield "normal-4x4x4-chi16-D256", g4, normal_tensors(g4, 0.1, seed=12), sweep_tree((4, 4, 4)), 16


CASES = list(_cases())


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES, ids=[c[0] for c in CASES])
def test_grad_matches_oracle_fp64(name, g, T, pairs, chi):
    print(f"\n[grad] {name}", flush=True)
    sign, lnz, grads, tie = gpu_grad(g, T, pairs, chi)
    if tie.any():
        pytest.skip("a truncation tie: several gradients are correct")
    ref = lnz_and_grad(g.n, g.edges, T, pairs, chi)
    assert sign == ref.sign
    assert lnz == pytest.approx(ref.ln_abs_z, rel=1e-10)
    scale = max(float(np.max(np.abs(r))) for r in ref.grads)
    worst = max(float(np.max(np.abs(a - r))) for a, r in zip(grads, ref.grads))
    assert worst <= GRAD_RTOL * scale, f"max |dg| = {worst:.3e}, max |g| = {scale:.3e}"


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES, ids=[c[0] for c in CASES])
def test_grad_euler_identity_gpu(name, g, T, pairs, chi):
    _, _, grads, _ = gpu_grad(g, T, pairs, chi)
    for t, gr in zip(T, grads):
        assert float(np.sum(t * gr)) == pytest.approx(1.0, abs=1e-10)


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES[:7], ids=[c[0] for c in CASES[:7]])
def test_grad_fp32_bound(name, g, T, pairs, chi):
    _, lnz, grads, tie = gpu_grad(g, T, pairs, chi, precision="fp32")
    if tie.any():
        pytest.skip("a truncation tie")
    ref = lnz_and_grad(g.n, g.edges, T, pairs, chi)
    scale = max(float(np.max(np.abs(r))) for r in ref.grads)
    worst = max(float(np.max(np.abs(a - r))) for a, r in zip(grads, ref.grads))
    print(f"fp32 grad {name}: max |dg| / max |g| = {worst / scale:.2e}", flush=True)
    assert worst <= FP32_GRAD_RTOL * scale


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES[:7], ids=[c[0] for c in CASES[:7]])
def test_grad_bf16_bound(name, g, T, pairs, chi):
    # bfloat16 tensors: every stored entry is rounded to 8 significant bits
    _, lnz, grads, tie = gpu_grad(g, T, pairs, chi, precision="bf16")
    if tie.any():
        pytest.skip("a truncation tie")
    ref = lnz_and_grad(g.n, g.edges, T, pairs, chi)
    scale = max(float(np.max(np.abs(r))) for r in ref.grads)
    worst = max(float(np.max(np.abs(a - r))) for a, r in zip(grads, ref.grads))
    print(f"bf16 grad {name}: max |dg| / max |g| = {worst / scale:.2e}", flush=True)
    assert worst <= 0.1 * scale


@pytest.mark.parametrize("shape,beta,seed,chi", [((3, 3), 0.44, None, 2), ((4, 4), 0.44, 4, 4),
                                                 ((2, 2, 3), 0.3, 5, 8), ((3, 4), 0.6, 3, 2)])
def test_coupling_gradient_exact_regime(shape, beta, seed, chi):
    g = lattice(shape)
    J = np.ones(g.n_edges) if seed is None else np.where(np.random.default_rng(seed).random(g.n_edges) < 0.5, -1.0, 1.0)
    T = ising_tensors(g, beta, J)
    _, lnz, grads, _ = gpu_grad(g, T, sweep_tree(shape), chi)
    assert lnz == pytest.approx(exact.ising_brute_force(g.n, g.edges, beta, J), rel=1e-12)
    dJ = ising_coupling_grad(g.n, g.edges, beta, J, grads)
    want = beta * exact.ising_correlations_brute(g.n, g.edges, beta, J)
    np.testing.assert_allclose(dJ, want, rtol=1e-9, atol=1e-12)


def test_grad_requires_grad_plan():
    g = lattice((3, 3))
    T = ising_tensors(g, 0.4)
    eu, ev, ed, off, data = flat(g, T)
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        p = sweep_tree((3, 3))
        c.tn_set_tree([a for a, _ in p], [b for _, b in p], 2)
        c.tn_contract_compressed()
        with pytest.raises(tn.TNError) as e:
            c.tn_grad()
        assert e.value.status == tn.TN_ESTATE
        c.tn_set_tree([a for a, _ in p], [b for _, b in p], 2, grad=True)
        with pytest.raises(tn.TNError) as e:
            c.tn_grad()          # planned for gradients but not evaluated yet
        assert e.value.status == tn.TN_ESTATE
    finally:
        c.close()
