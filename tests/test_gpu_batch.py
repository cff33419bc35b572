"""Batches: uneven instances merged level by level and replayed from one hipGraph.

A batch runs the same kernels on the same descriptors as the separate
evaluations, only grouped differently, so its results must be bitwise equal to
them; replays follow new values given between them (with eager work and
synchronisation in between), and the batched reverse pass equals tn_grad.
"""
import numpy as np
import pytest

import paper_2206_07044_amd as tn
import oracle
from tninputs import dimer_tensors, greedy_tree, ising_tensors, lattice, normal_tensors, random_regular3
from tninputs.trees import sweep_tree

pytestmark = pytest.mark.gpu


def flat(g, T):
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    return eu, ev, ed, off, np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T])


def instances():
    out = []
    for n, seed in ((40, 0), (60, 1), (80, 2), (100, 3)):        # uneven dimer instances (SI F.3)
        g = random_regular3(n, seed)
        out.append((g, dimer_tensors(g), greedy_tree(g, 8, seed), 8))
    g = lattice((6, 6))
    out.append((g, ising_tensors(g, 0.44), sweep_tree((6, 6)), 4))
    g = lattice((4, 4, 4))
    out.append((g, normal_tensors(g, 0.3, seed=5), sweep_tree((4, 4, 4)), 6))
    return out


def make_ctx(g, T, pairs, chi, precision="fp64", grad=False):
    eu, ev, ed, off, data = flat(g, T)
    c = tn.Context(0)
    c.tn_load_graph(g.n, eu, ev, ed, off, data)
    c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision, grad=grad)
    return c, off


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_bitwise_equal_to_separate_runs(precision):
    insts = instances()
    ctxs = [make_ctx(*i, precision=precision)[0] for i in insts]
    try:
        single = []
        for c in ctxs:
            c.tn_contract_compressed()
            single.append(c.tn_result())
        b = tn.Batch(ctxs)
        try:
            m, e = b.tn_batch_contract()
            for i, c in enumerate(ctxs):
                assert c.tn_result() == single[i], f"instance {i}"
                if precision == "fp64":
                    want = oracle.contract_compressed(insts[i][0].n, insts[i][0].edges, insts[i][1], insts[i][2],
                                                      insts[i][3])
                    assert single[i][1] == pytest.approx(want.ln_abs_z, rel=1e-10)
        finally:
            b.close()
    finally:
        for c in ctxs:
            c.close()


def test_batch_replays_follow_new_values():
    insts = instances()[:3] + instances()[4:5]
    ctxs = [make_ctx(*i)[0] for i in insts]
    b = tn.Batch(ctxs)
    try:
        rng = np.random.default_rng(0)
        for rep in range(3):
            # new values for every instance, eager work and synchronisation between replays
            datas = []
            for (g, T, pairs, chi), c in zip(insts, ctxs):
                T2 = [t * rng.uniform(0.5, 2.0) + (0.05 * rng.random(t.shape) if rep else 0.0) for t in T]
                datas.append((g, T2, pairs, chi))
                c.tn_update_values(flat(g, T2)[4])
            b.tn_batch_contract()
            got = [c.tn_result() for c in ctxs]
            for (g, T2, pairs, chi), r in zip(datas, got):
                e = tn.Context(0)
                try:
                    eu, ev, ed, off, data = flat(g, T2)
                    e.tn_load_graph(g.n, eu, ev, ed, off, data)
                    e.tn_set_tree([a for a, _ in pairs], [bb for _, bb in pairs], chi)
                    e.tn_contract_compressed()
                    assert e.tn_result() == r, f"replay {rep}"
                finally:
                    e.close()
    finally:
        b.close()
        for c in ctxs:
            c.close()


def test_batch_grad_equals_separate_grad():
    torch = pytest.importorskip("torch")
    insts = instances()[4:] + [instances()[0]]
    made = [make_ctx(*i, grad=True) for i in insts]
    ctxs = [m[0] for m in made]
    try:
        want = []
        for c in ctxs:
            c.tn_contract_compressed()
            want.append(c.tn_grad())
        b = tn.Batch(ctxs)
        try:
            outs = [torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda") for _, off in made]
            for rep in range(2):
                b.tn_batch_contract()
                b.tn_batch_grad([o.data_ptr() for o in outs])
                for i, o in enumerate(outs):
                    np.testing.assert_array_equal(o.cpu().numpy(), want[i])
                    o.zero_()
                    torch.cuda.synchronize()
        finally:
            b.close()
    finally:
        for c in ctxs:
            c.close()


def test_batch_rejects_mixed_precision():
    insts = instances()
    a = make_ctx(*insts[0], precision="fp64")[0]
    c = make_ctx(*insts[1], precision="fp32")[0]
    try:
        with pytest.raises(tn.TNError) as e:
            tn.Batch([a, c])
        assert e.value.status == tn.TN_EINVAL
    finally:
        a.close()
        c.close()
