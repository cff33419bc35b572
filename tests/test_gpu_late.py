"""Late compression (section II.D; Algorithm 1 with compress_late): before contracting i and j,
every other bond of i, then of j, larger than chi is compressed.  GPU against the oracle's late
schedule: ln|Z| in FP64 at 1e-10 relative on lattices, random graphs and the URand model of the
paper's early-versus-late comparison (D = 4 square lattice, entries in [-0.5, 1]), and the
reverse pass element by element at 1e-9 of the largest |g|."""
import numpy as np
import pytest

import paper_2206_07044_amd as tn
from oracle.grad import lnz_and_grad
from tninputs import configs, ising_tensors, lattice, normal_tensors, uniform_tensors
from tninputs.trees import sweep_tree

from test_gpu_parity import _check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("chi", [2, 4, 8])
def test_late_ising_8x8(chi):
    g = lattice((8, 8))
    _check(g, ising_tensors(g, 0.44), sweep_tree((8, 8)), chi, min_comp=1, late=True)


@pytest.mark.parametrize("shape,chi", [((4, 4, 4), 8), ((5, 5, 5), 8), ((4, 4, 4), 16)])
def test_late_ising_cubic(shape, chi):
    g = lattice(shape)
    _check(g, ising_tensors(g, 0.22), sweep_tree(shape), chi, min_comp=1, late=True)


@pytest.mark.parametrize("L,chi,seed", [(6, 8, 0), (6, 16, 1), (8, 8, 2)])
def test_late_urand_square_d4(L, chi, seed):
    g = lattice((L, L), dim=4)
    _check(g, uniform_tensors(g, -0.5, seed), sweep_tree((L, L)), chi, min_comp=1, late=True)


def test_late_random_graphs():
    g, T, pairs = configs.dimer_rrg(200, 4)
    _check(g, T, pairs, 4, min_comp=20, late=True)
    g, T, pairs = configs.normal_rrg(100, 0.2, 2, tensor_seed=1)
    _check(g, T, pairs, 2, min_comp=20, late=True)


@pytest.mark.parametrize("case", ["pmJ-4x4x4-chi4", "ising-8x8-chi4", "normal-4x4x4-chi6"])
def test_late_gradient_matches_oracle(case):
    if case == "pmJ-4x4x4-chi4":
        g = lattice((4, 4, 4))
        J = np.where(np.random.default_rng(9).random(g.n_edges) < 0.5, -1.0, 1.0)
        T, pairs, chi = ising_tensors(g, 0.5, J), sweep_tree((4, 4, 4)), 4
    elif case == "ising-8x8-chi4":
        g = lattice((8, 8))
        T, pairs, chi = ising_tensors(g, 0.44), sweep_tree((8, 8)), 4
    else:
        g = lattice((4, 4, 4))
        T, pairs, chi = normal_tensors(g, 0.3, seed=3), sweep_tree((4, 4, 4)), 6
    want = lnz_and_grad(g.n, g.edges, T, pairs, chi, compress_late=True)
    eu, ev, ed = g.arrays()
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, np.concatenate([t.ravel() for t in T]))
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, grad=True, late=True)
        c.tn_contract_compressed()
        sign, lnz = c.tn_result()
        gflat = c.tn_grad()
        _, tie, _ = c.tn_compress_stats()
    finally:
        c.close()
    if tie.any():
        pytest.skip("truncation tie")
    scale = max(float(np.max(np.abs(x))) for x in want.grads)
    err = max(float(np.max(np.abs(gflat[off[v]:off[v + 1]] - want.grads[v].ravel()))) for v in range(g.n))
    print(f"late {case}: lnZ {lnz!r} oracle {want.ln_abs_z!r}; max|g - oracle| {err:.2e} (max|g| {scale:.2e})",
          flush=True)
    assert sign == want.sign and abs(lnz - want.ln_abs_z) <= 1e-10 * abs(want.ln_abs_z)
    assert err <= 1e-9 * scale
