"""GEMM tile table and its autotuner on the GPU.

Every tile computes the same product, so whichever table is installed when a tree is planned,
ln Z and the gradient must agree with the oracle (and with each other up to summation order).
The tables tried force every class onto one family: all 64 x 64 MFMA, every skinny-kernel tile
where it applies (including the 32-wide ones the defaults do not take), every MFMA skinny tile,
and the autotuner's own choice.
"""
import functools

import numpy as np
import pytest

import paper_2206_07044_amd as tn
from paper_2206_07044_amd import autotune
from oracle.approx import contract_compressed
from oracle.grad import lnz_and_grad
from tninputs import ising_tensors, lattice, normal_tensors
from tninputs.configs import pm_couplings
from tninputs.trees import sweep_tree

pytestmark = pytest.mark.gpu

FAMILIES = {
    "mfma64": [0],
    "skinny": [5, 6, 7, 8, 0],
    "mfma_skinny": [1, 2, 3, 4, 0],
}


def _allowed(klass, tile):
    k = (klass // 2) % 3
    short32 = (klass // 6) % 2
    wide = (klass // 12) % 2
    if tile == 0:
        return True
    tall = {1: not short32, 3: True, 5: not short32 and k <= 1, 6: k <= 1}
    wid = {2: not short32, 4: True, 7: not short32 and k <= 1, 8: k <= 1}
    return (wid if wide else tall).get(tile, False)


def family_table(prefs):
    return np.array([next(t for t in prefs if _allowed(c, t)) for c in range(tn.GEMM_CLASSES)], dtype=np.int32)


@pytest.fixture(autouse=True)
def restore_table():
    yield
    tn.tn_gemm_tiles_set(None)


def flat(g, T):
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    return eu, ev, ed, off, np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T])


def run(g, T, pairs, chi, precision, grad=False):
    eu, ev, ed, off, data = flat(g, T)
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision, grad=grad)
        c.tn_contract_compressed()
        lnz = c.tn_result()[1]
        return lnz, (c.tn_grad() if grad else None)
    finally:
        c.close()


def test_tune_measures_the_allowed_tiles():
    for klass in (autotune.class_of(1, False, False, 1, True), autotune.class_of(0, True, True, 0, True),
                  autotune.class_of(2, True, False, 2, False)):
        us = tn.tn_gemm_tune(klass, copies=2)
        print(autotune.describe(klass), {tn.GEMM_TILES[t]: round(float(us[t]), 1) for t in range(9) if us[t] > 0},
              flush=True)
        for t in range(9):
            assert (us[t] > 0) == _allowed(klass, t), (klass, t, us[t])


def test_autotuner_installs_the_fastest_tiles():
    report = autotune.tune(precisions=("fp32",), copies=4)
    table = tn.tn_gemm_tiles_get()
    assert len(report["timings_us"]) == 24
    for c in autotune.classes_of(("fp32",)):
        times = report["timings_us"][autotune.describe(c)]
        assert tn.GEMM_TILES[table[c]] == min(times, key=times.get)
    print(f"tuned 24 classes in {report['seconds']:.2f} s; changed {report['changed']}", flush=True)


@functools.lru_cache(maxsize=None)
def cases():
    """(graph, tensors, tree, chi) and the oracle's ln|Z| (and gradient) for each, computed once."""
    g = lattice((6, 6, 6))
    T = ising_tensors(g, 0.5, pm_couplings(g.n_edges, 0))
    pairs = sweep_tree((6, 6, 6))
    g5 = lattice((5, 5, 4))
    T5 = ising_tensors(g5, 0.25)
    p5 = sweep_tree((5, 5, 4))
    g4 = lattice((4, 4, 4))
    T4 = normal_tensors(g4, 0.1, seed=12)
    p4 = sweep_tree((4, 4, 4))
    r4 = lnz_and_grad(g4.n, g4.edges, T4, p4, 16)
    return ((g, T, pairs, contract_compressed(g.n, g.edges, T, pairs, 8).ln_abs_z),
            (g5, T5, p5, contract_compressed(g5.n, g5.edges, T5, p5, 32).ln_abs_z),
            (g4, T4, p4, r4.ln_abs_z, np.concatenate([x.ravel() for x in r4.grads])))


@pytest.mark.parametrize("family", sorted(FAMILIES))
def test_every_tile_family_matches_the_oracle(family):
    tn.tn_gemm_tiles_set(family_table(FAMILIES[family]))
    (g, T, pairs, ref), (g5, T5, p5, ref5), (g4, T4, p4, ref4, refg) = cases()
    lnz, _ = run(g, T, pairs, 8, "fp64")
    assert abs(lnz - ref) <= 1e-10 * abs(ref)
    lnz32, _ = run(g, T, pairs, 8, "fp32")
    assert abs(lnz32 - ref) <= 2e-6 * abs(ref)
    # chi = 32 (32-wide classes), forward
    lnz5, _ = run(g5, T5, p5, 32, "fp64")
    assert abs(lnz5 - ref5) <= 1e-10 * abs(ref5)
    # D = 256 cores with the reverse pass (adjoint GEMMs take the table too)
    lnz4, grad4 = run(g4, T4, p4, 16, "fp64", grad=True)
    assert abs(lnz4 - ref4) <= 1e-10 * abs(ref4)
    assert np.max(np.abs(grad4 - refg)) <= 1e-9 * np.max(np.abs(refg))
