"""Tree-gauge compression (r >= 1; section II.C, SI A): the R factors of each compression come
from the bond placed in the tree gauge of the r-local spanning tree around it, computed on the GPU
as environment metrics.  FP64 against the oracle (which gauges virtual copies by inward QR) at
1e-10 relative, with early and late compression; the probe whose environment is rank 1, exact at
chi = 2 only through the gauge; FP32 at the random-walk bound; gradient plans refuse r >= 1."""
import math

import numpy as np
import pytest

import oracle
import paper_2206_07044_amd as tn
from tninputs import configs, ising_tensors, lattice, normal_tensors, uniform_tensors
from tninputs.trees import sweep_tree

from _gpu_helpers import gpu_eval
from test_gpu_parity import FP64_RTOL, _fp32_bound

pytestmark = pytest.mark.gpu


def _gauge_check(g, T, pairs, chi, r, late=False, precision="fp64", min_comp=1):
    want = oracle.contract_compressed(g.n, g.edges, T, pairs, chi, gauge_r=r, compress_late=late)
    comp = [o for o in want.ops if o.kind == "compress"]
    print(f"gauge r={r} late={late} n={g.n} chi={chi} {precision}: oracle {want.ln_abs_z!r}, "
          f"{len(comp)} compressions", flush=True)
    assert len(comp) >= min_comp
    if any(o.tie for o in comp):
        pytest.skip("truncation tie in the oracle run")
    eu, ev, ed = g.arrays()
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, np.concatenate([t.ravel() for t in T]))
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision, late=late, gauge_r=r)
        c.tn_contract_compressed()
        sign, lnz = c.tn_result()
    finally:
        c.close()
    err = abs(lnz - want.ln_abs_z)
    print(f"    gpu {lnz!r}, |d lnZ| {err:.3e}", flush=True)
    assert sign == want.sign
    bound = FP64_RTOL * max(1.0, abs(want.ln_abs_z)) if precision == "fp64" else _fp32_bound(want)
    assert err <= bound
    return want, lnz


def test_rank1_environment_is_exact_only_with_the_gauge():
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_pins import _rank1_environment_network
    g, T, pairs = _rank1_environment_network()
    ex = oracle.contract_compressed(g.n, g.edges, T, pairs, None)
    _, lnz1 = _gauge_check(g, T, pairs, 2, 1)
    assert abs(lnz1 - ex.ln_abs_z) <= 1e-12 * max(1.0, abs(ex.ln_abs_z))
    sign0, lnz0, *_ = gpu_eval(g, T, pairs, 2)
    assert abs(lnz0 - ex.ln_abs_z) > 1e-3


@pytest.mark.parametrize("r", [1, 2, 4])
@pytest.mark.parametrize("late", [False, True])
def test_gauge_urand_square_d4(r, late):
    g = lattice((8, 8), dim=4)
    _gauge_check(g, uniform_tensors(g, -0.5, 0), sweep_tree((8, 8)), 8, r, late)


@pytest.mark.parametrize("case", ["ising-4x4x4-chi8-r2", "pmJ-5x5x5-chi8-r1", "pmJ-5x5x5-chi8-r3",
                                  "normal-4x4x4-chi16-r2-D256", "dimer-rrg200-chi4-r2"])
def test_gauge_lattices_and_graphs(case):
    if case.startswith("ising"):
        g = lattice((4, 4, 4))
        _gauge_check(g, ising_tensors(g, 0.22), sweep_tree((4, 4, 4)), 8, 2)
    elif case.startswith("pmJ"):
        g = lattice((5, 5, 5))
        T = ising_tensors(g, 0.5, configs.pm_couplings(g.n_edges, 0))
        _gauge_check(g, T, sweep_tree((5, 5, 5)), 8, int(case[-1]))
    elif case.startswith("normal"):
        g = lattice((4, 4, 4))   # the last sweep stage merges two chi-bonds: D = 256 on the block-Jacobi core
        _gauge_check(g, normal_tensors(g, 0.3, seed=3), sweep_tree((4, 4, 4)), 16, 2)
    else:
        g, T, pairs = configs.dimer_rrg(200, 4)
        _gauge_check(g, T, pairs, 4, 2, min_comp=20)


def test_gauge_fp32():
    g = lattice((4, 4, 4))
    _gauge_check(g, ising_tensors(g, 0.22), sweep_tree((4, 4, 4)), 8, 2, precision="fp32")


def test_gauge_refuses_gradient_plans():
    g = lattice((3, 3))
    T = ising_tensors(g, 0.44)
    eu, ev, ed = g.arrays()
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    pairs = sweep_tree((3, 3))
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, np.concatenate([t.ravel() for t in T]))
        with pytest.raises(tn.TNError) as e:
            c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], 2, grad=True, gauge_r=1)
        assert e.value.status == tn.TN_EINVAL
    finally:
        c.close()
