"""R-factors by batched Householder TSQR (tn_tree_opts.r_factor = TN_RFACTOR_TSQR).

Section II.C forms each bond's reduced factors by QR of the two matricised sides, as the oracle
does with LAPACK.  The library's default takes them from float64 Grams (pivoted Cholesky); the
TSQR option reduces row blocks in LDS by Householder reflections and then the stacked R's.
Checked here: ln Z against the oracle on lattices, random graphs and a spin glass (FP64 at the
1e-10 bar, FP32 near its rounding level), a bond whose sides need several TSQR passes, and the
one-bond probe of the Gram route's accuracy floor, where TSQR keeps the directions below 3e-8 of
the largest that the Gram route drops.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2206_07044_amd as tn
from tninputs import dimer_tensors, ising_tensors, lattice, normal_tensors, random_regular3
from tninputs.configs import pm_couplings
from tninputs.trees import agglom_tree, sweep_tree

pytestmark = pytest.mark.gpu


def run(g, T, pairs, chi, precision="fp64", r_factor="tsqr"):
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    data = np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T])
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision, r_factor=r_factor)
        m, _ = c.tn_contract_compressed()
        return c.tn_result() if m != 0.0 else (0.0, -math.inf)
    finally:
        c.close()


def _cases():
    g6 = lattice((6, 6, 6))
    yield "pmJ-6x6x6-chi8", g6, ising_tensors(g6, 0.5, pm_couplings(g6.n_edges, 0)), sweep_tree((6, 6, 6)), 8
    g4 = lattice((4, 4, 4))
    yield "normal-4x4x4-chi6", g4, normal_tensors(g4, 0.3, seed=3), sweep_tree((4, 4, 4)), 6
    g8 = lattice((8, 8))
    yield "ising-8x8-chi8", g8, ising_tensors(g8, 0.44), sweep_tree((8, 8)), 8
    rr = random_regular3(40, seed=0)
    yield "dimer-rrg40-chi4", rr, dimer_tensors(rr), agglom_tree(rr, 4, seed=0), 4
    g3 = lattice((5, 5), dim=3)
    yield "normal-5x5-D3-chi5", g3, normal_tensors(g3, 0.2, seed=1), sweep_tree((5, 5)), 5


CASES = list(_cases())


@pytest.mark.parametrize("name,g,T,pairs,chi", CASES, ids=[c[0] for c in CASES])
def test_tsqr_matches_the_oracle(name, g, T, pairs, chi):
    want = oracle.contract_compressed(g.n, g.edges, T, pairs, chi)
    comp = [o for o in want.ops if o.kind == "compress"]
    assert comp, "the case does not compress"
    if any(o.tie for o in comp):
        pytest.skip("a truncation tie in the oracle run: several values are correct")
    sign, lnz = run(g, T, pairs, chi, "fp64")
    rel = abs(lnz - want.ln_abs_z) / max(1.0, abs(want.ln_abs_z))
    gram = run(g, T, pairs, chi, "fp64", "gram")[1]
    print(f"{name}: tsqr {lnz!r}, gram {gram!r}, oracle {want.ln_abs_z!r}, rel {rel:.2e}, "
          f"{len(comp)} compressions", flush=True)
    assert sign == want.sign and rel <= 1e-10
    sign32, lnz32 = run(g, T, pairs, chi, "fp32")
    assert sign32 == want.sign and abs(lnz32 - want.ln_abs_z) <= 2e-6 * max(1.0, abs(want.ln_abs_z))


def test_tsqr_several_passes():
    """12^3 tree prefix bonds have sides of up to 2^17 rows: pass 0 blocks of 512 rows (D = 32),
    then the stacked R's; the full tree at chi = 16 against the grouped Gram route and the
    stored oracle value."""
    import json
    import os
    g = lattice((12, 12, 12))
    T = ising_tensors(g, 0.22)
    pairs = sweep_tree((12, 12, 12))
    sign, lnz = run(g, T, pairs, 16, "fp64")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cubic_12.json")))
    ref = float(gold["oracle_lnZ"])
    print(f"12^3 chi=16 tsqr: {lnz!r}, oracle {ref!r}, rel {abs(lnz - ref) / ref:.2e}", flush=True)
    # the instance's own rounding band (the oracle spreads over 4e-7 with its BLAS thread count)
    assert sign == 1.0 and abs(lnz - ref) <= 1e-6 * ref


@pytest.mark.parametrize("s_small", [[1e-9, 1e-11], [1e-6, 1e-10], [1e-7, 1e-7]])
def test_tsqr_keeps_what_the_gram_route_drops(s_small):
    """The one-bond probe of the Gram-route floor (a side of rank 6 with singular values down to
    1e-11 of its largest, chi = 6, nothing truncated): TSQR's R keeps every direction, so Z is
    right up to the rounding of well-conditioned Householder steps."""
    from tninputs.probes import bond_probe
    rng = np.random.default_rng(31)
    s_a = np.array([1.0, 1e-2, 1e-5, 1e-6] + s_small + [0.0, 0.0])
    ua, _ = np.linalg.qr(rng.normal(size=(12, 8)))
    va, _ = np.linalg.qr(rng.normal(size=(8, 8)))
    a_mat = (ua * s_a) @ va.T
    b_mat = rng.normal(size=(8, 12))
    caps = [rng.normal(size=d) + 1.0 for d in (3, 4, 3, 4)]
    g, T, pairs = bond_probe(a_mat, b_mat, (2, 4), (3, 4), (3, 4), caps)
    z = np.kron(caps[0], caps[1]) @ a_mat @ b_mat @ np.kron(caps[2], caps[3])
    small = (s_a > 0) & (s_a < 3.2e-8 * s_a[0])
    carried = abs(np.kron(caps[0], caps[1]) @ ((ua * np.where(small, s_a, 0.0)) @ va.T) @ b_mat
                  @ np.kron(caps[2], caps[3]))
    sign, lnz = run(g, T, pairs, 6, "fp64")
    sign_g, lnz_g = run(g, T, pairs, 6, "fp64", "gram")
    err = abs(sign * math.exp(lnz) - z)
    err_g = abs(sign_g * math.exp(lnz_g) - z)
    print(f"floor probe {s_small}: |Z - z| tsqr {err:.3e}, gram {err_g:.3e}, dropped part {carried:.3e}, "
          f"|z| {abs(z):.3e}", flush=True)
    assert sign == np.sign(z)
    assert err <= 1e-12 * abs(z)
    if carried > 0:
        assert err <= 1e-3 * carried <= err_g


def test_tsqr_option_errors():
    g = lattice((3, 3))
    T = ising_tensors(g, 0.4)
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    data = np.concatenate([t.ravel() for t in T])
    pairs = sweep_tree((3, 3))
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        with pytest.raises(tn.TNError) as e:
            c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], 2, grad=True, r_factor="tsqr")
        assert e.value.status == tn.TN_EINVAL
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], 2, r_factor="tsqr")
        with pytest.raises(tn.TNError) as e:
            tn.Batch([c])
        assert e.value.status == tn.TN_EINVAL
    finally:
        c.close()
