"""Ising coupling map on the GPU and the torch.autograd bindings.

The coupling map is checked against the seeded input generator; d ln Z / d J
through torch.autograd against the oracle's reference gradient and its
coupling chain, against brute-force spin correlations in the exact regime, and
against central finite differences (h = 1e-5, FP64 forward) on sampled bonds
of a reduced frustrated 3D instance (6^3, +-J, beta = 0.5).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2206_07044_amd as tn  # noqa: E402
from oracle import exact  # noqa: E402
from oracle.grad import ising_coupling_grad, lnz_and_grad  # noqa: E402
from tninputs import ising_tensors, lattice, normal_tensors  # noqa: E402
from tninputs.trees import sweep_tree  # noqa: E402

pytestmark = pytest.mark.gpu


def pm_couplings(n_edges, seed):
    return np.where(np.random.default_rng(seed).random(n_edges) < 0.5, -1.0, 1.0)


def test_ising_values_match_generator():
    from paper_2206_07044_amd.autograd import IsingLogZ
    g = lattice((3, 4))
    J = pm_couplings(g.n_edges, 1) * np.linspace(0.5, 1.5, g.n_edges)
    net = IsingLogZ(g.n, g.edges, sweep_tree((3, 4)), 4, beta=0.7)
    try:
        Jt = torch.tensor(J, dtype=torch.float64, device="cuda")
        net.ctx.tn_ising_values_device(0.7, Jt.data_ptr())
        net.ctx.tn_contract_compressed()
        # the evaluation read the GPU-built tensors: compare them entry by entry
        want = ising_tensors(g, 0.7, J)
        for v in range(g.n):
            got = net.ctx.tn_read_tensor(v)
            np.testing.assert_allclose(got, (want[v] / np.max(np.abs(want[v]))).ravel(), rtol=1e-14, atol=1e-15)
    finally:
        net.close()


@pytest.mark.parametrize("shape,beta,chi,seed", [((4, 4), 0.5, 2, 7), ((2, 2, 3), 0.5, 3, 3), ((6, 6, 6), 0.5, 8, 0)])
def test_autograd_coupling_gradient_matches_oracle(shape, beta, chi, seed):
    from paper_2206_07044_amd.autograd import IsingLogZ
    print(f"\n[autograd] {shape} chi={chi}", flush=True)
    g = lattice(shape)
    J = pm_couplings(g.n_edges, seed)
    pairs = sweep_tree(shape)
    net = IsingLogZ(g.n, g.edges, pairs, chi, beta)
    try:
        Jt = torch.tensor(J, dtype=torch.float64, device="cuda", requires_grad=True)
        lnz = net(Jt)
        lnz.backward()
        got = Jt.grad.cpu().numpy()
    finally:
        net.close()
    ref = lnz_and_grad(g.n, g.edges, ising_tensors(g, beta, J), pairs, chi)
    assert float(lnz.detach()) == pytest.approx(ref.ln_abs_z, rel=1e-10)
    want = ising_coupling_grad(g.n, g.edges, beta, J, ref.grads)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9 * np.max(np.abs(want)))


def test_autograd_exact_regime_spin_correlations():
    from paper_2206_07044_amd.autograd import IsingLogZ
    g = lattice((4, 4))
    J = pm_couplings(g.n_edges, 4)
    net = IsingLogZ(g.n, g.edges, sweep_tree((4, 4)), 4, beta=0.44)   # exact compressions
    try:
        Jt = torch.tensor(J, dtype=torch.float64, device="cuda", requires_grad=True)
        net(Jt).backward()
        got = Jt.grad.cpu().numpy()
    finally:
        net.close()
    want = 0.44 * exact.ising_correlations_brute(g.n, g.edges, 0.44, J)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12)


def test_autograd_central_differences_sampled_bonds():
    from paper_2206_07044_amd.autograd import IsingLogZ
    shape, beta, chi, h = (6, 6, 6), 0.5, 8, 1e-5
    g = lattice(shape)
    J = pm_couplings(g.n_edges, 0)
    net = IsingLogZ(g.n, g.edges, sweep_tree(shape), chi, beta)
    try:
        Jt = torch.tensor(J, dtype=torch.float64, device="cuda", requires_grad=True)
        net(Jt).backward()
        grad = Jt.grad.cpu().numpy()
        bonds = np.random.default_rng(12).choice(g.n_edges, size=12, replace=False)
        for e in bonds:
            Jp, Jm = J.copy(), J.copy()
            Jp[e] += h
            Jm[e] -= h
            with torch.no_grad():
                fp = float(net(torch.tensor(Jp, dtype=torch.float64, device="cuda")))
                fm = float(net(torch.tensor(Jm, dtype=torch.float64, device="cuda")))
            assert grad[e] == pytest.approx((fp - fm) / (2 * h), rel=1e-5, abs=1e-8), f"bond {e}"
    finally:
        net.close()


def test_tensor_logz_autograd_euler():
    from paper_2206_07044_amd.autograd import TensorLogZ
    g = lattice((3, 3), dim=3)
    T = normal_tensors(g, 0.2, seed=1)
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    data = np.concatenate([t.ravel() for t in T])
    f = TensorLogZ(g.n, g.edges, off, sweep_tree((3, 3)), 2)
    try:
        x = torch.tensor(data, dtype=torch.float64, device="cuda", requires_grad=True)
        f(x).backward()
        gr = x.grad.cpu().numpy()
    finally:
        f.close()
    for v in range(g.n):
        assert float(np.dot(data[off[v]:off[v + 1]], gr[off[v]:off[v + 1]])) == pytest.approx(1.0, abs=1e-10)
    ref = lnz_and_grad(g.n, g.edges, T, sweep_tree((3, 3)), 2)
    np.testing.assert_allclose(gr, np.concatenate([r.ravel() for r in ref.grads]), rtol=0,
                               atol=1e-9 * max(np.max(np.abs(r)) for r in ref.grads))
