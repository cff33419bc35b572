"""C-ABI behaviour on the GPU: caller-owned workspace, the plan budget, the state
left by a failed evaluation, and autograd over a shared context."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2206_07044_amd as tn  # noqa: E402
from paper_2206_07044_amd._capi import TNError, TN_ENOMEM, TN_EINVAL, TN_ENUMERIC, TN_ESTATE  # noqa: E402
from tninputs import ising_tensors, lattice  # noqa: E402
from tninputs.trees import sweep_tree  # noqa: E402

pytestmark = pytest.mark.gpu


def _load(c, g, T):
    eu, ev, ed = g.arrays()
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    c.tn_load_graph(g.n, eu, ev, ed, off, np.concatenate([t.ravel() for t in T]))


def _pairs(shape):
    p = sweep_tree(shape)
    return [a for a, _ in p], [b for _, b in p]


def test_workspace_arena_matches_library_arena():
    shape, chi = (5, 5, 5), 8
    g = lattice(shape)
    T = ising_tensors(g, 0.22)
    pi, pj = _pairs(shape)
    c = tn.Context(0)
    try:
        _load(c, g, T)
        c.tn_set_tree(pi, pj, chi)
        need = c.tn_plan_info()["arena_bytes"]
        ref = c.tn_contract_compressed()
        ws = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        c.tn_set_workspace(ws.data_ptr(), ws.numel())
        c.tn_set_tree(pi, pj, chi)
        got = c.tn_contract_compressed()
        assert got == ref                              # same plan, same kernels: bitwise equal
        # too small: refused by the plan check before any launch
        c.tn_set_workspace(ws.data_ptr(), need // 2)
        with pytest.raises(TNError) as ei:
            c.tn_set_tree(pi, pj, chi)
        assert ei.value.status == TN_ENOMEM
        # misaligned
        with pytest.raises(TNError) as ei:
            c.tn_set_workspace(ws.data_ptr() + 8, 1024)
        assert ei.value.status == TN_EINVAL
        # back to library memory
        c.tn_set_workspace(None, 0)
        c.tn_set_tree(pi, pj, chi)
        assert c.tn_contract_compressed() == ref
    finally:
        c.close()


def test_device_budget_refuses_plan():
    shape = (4, 4, 4)
    g = lattice(shape)
    pi, pj = _pairs(shape)
    c = tn.Context(0)
    try:
        _load(c, g, ising_tensors(g, 0.22))
        c.tn_set_tree(pi, pj, 8)
        need = c.tn_plan_info()["arena_bytes"]
        with pytest.raises(TNError) as ei:
            c.tn_set_tree(pi, pj, 8, budget=need - 1)
        assert ei.value.status == TN_ENOMEM
        with pytest.raises(TNError) as ei:     # no plan is left behind
            c.tn_contract_compressed()
        assert ei.value.status == TN_ESTATE
        c.tn_set_tree(pi, pj, 8, budget=need)
        c.tn_contract_compressed()
    finally:
        c.close()


def test_failed_evaluation_leaves_no_result():
    """A Jacobi capped at one sweep does not converge: TN_ENUMERIC, and neither tn_result nor
    tn_grad may then read the failed evaluation."""
    shape = (4, 4, 4)
    g = lattice(shape)
    pi, pj = _pairs(shape)
    c = tn.Context(0)
    try:
        _load(c, g, ising_tensors(g, 0.22))
        c.tn_set_tree(pi, pj, 4, max_sweeps=1, grad=True)
        with pytest.raises(TNError) as ei:
            c.tn_contract_compressed()
        assert ei.value.status == TN_ENUMERIC
        for call in (c.tn_result, c.tn_grad):
            with pytest.raises(TNError) as ei:
                call()
            assert ei.value.status == TN_ESTATE
    finally:
        c.close()


def test_autograd_backward_after_a_second_forward():
    """Two forward passes on one planned context, then backward of the first: the context
    holds the second evaluation, so the first is recomputed before its reverse pass."""
    from paper_2206_07044_amd.autograd import IsingLogZ
    shape, chi, beta = (4, 4, 4), 4, 0.5
    g = lattice(shape)
    rng = np.random.default_rng(3)
    J1 = np.where(rng.random(g.n_edges) < 0.5, -1.0, 1.0)
    J2 = J1 * rng.uniform(0.5, 1.5, g.n_edges)
    pairs = sweep_tree(shape)
    net = IsingLogZ(g.n, g.edges, pairs, chi, beta)
    try:
        a = torch.tensor(J1, dtype=torch.float64, device="cuda", requires_grad=True)
        b = torch.tensor(J2, dtype=torch.float64, device="cuda", requires_grad=True)
        la = net(a)
        lb = net(b)
        la.backward()
        ga = a.grad.cpu().numpy()
        lb.backward()
        gb = b.grad.cpu().numpy()
        # references: one forward + backward each
        a2 = torch.tensor(J1, dtype=torch.float64, device="cuda", requires_grad=True)
        net(a2).backward()
        b2 = torch.tensor(J2, dtype=torch.float64, device="cuda", requires_grad=True)
        net(b2).backward()
    finally:
        net.close()
    np.testing.assert_array_equal(ga, a2.grad.cpu().numpy())
    np.testing.assert_array_equal(gb, b2.grad.cpu().numpy())
    assert not np.allclose(ga, gb)
    want = oracle.contract_compressed(g.n, g.edges, ising_tensors(g, beta, J1), pairs, chi)
    assert abs(la.item() - want.ln_abs_z) < 1e-10 * abs(want.ln_abs_z)


@pytest.mark.parametrize("shape,chi,precision", [((5, 5, 5), 8, "fp64"), ((8, 8), 16, "fp64"), ((6, 6, 6), 16, "fp64"),
                                                 ((4, 4, 4), 8, "fp32")])
def test_plain_form_equals_grouped_form(shape, chi, precision):
    """The plain form (one launch per step, one stream, no graph) runs the same kernels on the
    same descriptors as the grouped, captured form, so its result is bitwise the same."""
    g = lattice(shape)
    T = ising_tensors(g, 0.22 if len(shape) == 3 else 0.44)
    pi, pj = _pairs(shape)
    c = tn.Context(0)
    try:
        _load(c, g, T)
        c.tn_set_tree(pi, pj, chi, precision=precision)
        ref = c.tn_contract_compressed()
        c.tn_set_tree(pi, pj, chi, precision=precision, plain=True)
        got = [c.tn_contract_compressed() for _ in range(2)]
        assert got[0] == ref and got[1] == ref
        with pytest.raises(TNError) as ei:
            c.tn_set_tree(pi, pj, chi, plain=True, grad=True)
        assert ei.value.status == TN_EINVAL
        c.tn_set_tree(pi, pj, chi, precision=precision, plain=True)
        with pytest.raises(TNError) as ei:
            tn.Batch([c])
        assert ei.value.status == TN_EINVAL
    finally:
        c.close()
